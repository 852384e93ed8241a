"""26-qubit states (512 MiB complex64, 1 GiB complex128 each), the random
U3 + CZ layered workload with depolarizing noise.

* All 26 qubits, one layer: per-shot registers equal the FP64 oracle's.
* All 80 layers, shot ids 1000.. of the 2000-shot job: properties that
  hold at any size. Batch and branch modes give the same registers;
  the FP64 batch executor and the plain per-op FP64 form give the same
  registers; the complex64 and complex128 states of one trajectory agree
  to within complex64 rounding.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_run, mismatches, oracle_memory, say

pytestmark = pytest.mark.gpu

OFFSET = 1000


def _c4(layers):
    return (W.random_layered(26, layers, seed=0, two_qubit="cz"),
            W.depol_model(gates2=("cz",)))


def test_c4_qubits_one_layer_matches_oracle():
    circ, noise = _c4(1)
    shots = 3
    say("case c4 26q x 1 layer, c128 vs oracle")
    got = gpu_run(circ, noise, shots, dtype="c128", seed=0)
    exp = oracle_memory(circ, noise, shots, seed=0)
    assert mismatches(got["memory"], exp) == 0


def test_c4_full_depth_batch_equals_branch_c64():
    circ, noise = _c4(80)
    shots = 8
    say("case c4 26q x 80 layers, c64 batch vs branch, 8 shots")
    a = gpu_run(circ, noise, shots, dtype="c64", seed=0, shot_offset=OFFSET)
    b = gpu_run(circ, noise, shots, dtype="c64", mode="branch", seed=0, shot_offset=OFFSET)
    assert mismatches(a["memory"], b["memory"]) == 0


def test_c4_full_depth_executor_equals_plain_form_c128():
    circ, noise = _c4(80)
    shots = 2
    say("case c4 26q x 80 layers, c128 batch vs plain, 2 shots")
    a = gpu_run(circ, noise, shots, dtype="c128", seed=0, shot_offset=OFFSET)
    p = gpu_run(circ, noise, shots, dtype="c128", mode="plain", seed=0, shot_offset=OFFSET)
    assert mismatches(a["memory"], p["memory"]) == 0


def test_c4_full_depth_c64_state_agrees_with_c128():
    circ, noise = _c4(80)
    say("case c4 26q x 80 layers, c64 vs c128 state of one shot")
    a = gpu_run(circ, noise, 1, dtype="c64", seed=0, shot_offset=OFFSET, dump_shot=0)
    b = gpu_run(circ, noise, 1, dtype="c128", seed=0, shot_offset=OFFSET, dump_shot=0)
    sa, sb = a["state"], b["state"]
    assert abs(np.vdot(sb, sb).real - 1.0) < 1e-9
    # ~6000 complex64 ops at 2^-24 relative rounding each: amplitude error
    # well below 1e-3 in norm, so infidelity below 1e-6
    fid = abs(np.vdot(sa, sb)) ** 2 / (np.vdot(sa, sa).real * np.vdot(sb, sb).real)
    say(f"c64/c128 fidelity 1-{1 - fid:.3e}, max |d amp| {np.max(np.abs(sa - sb)):.3e}")
    assert fid > 1 - 1e-6
    del sa, sb
