"""States that live in LDS for the whole shot (10 to 13 qubits) with the
register-group engine (option engine=2): their gates run in register groups
of n - 8 qubits, where each thread gathers 2^(n-8) amplitudes, applies the
group's fused micro-ops in registers and scatters them back. The per-shot registers must equal the FP64 oracle's (complex128)
in batch and branch mode, with Kraus and Pauli noise, mid-circuit measures,
conditional ops and dense multi-qubit ops; the kept state must equal the
oracle's amplitudes."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import dm
from gpu_util import gpu_run, mismatches, oracle_memory, say

pytestmark = pytest.mark.gpu


def _noise():
    return W.noise_model(
        [W.rule(["u3", "h", "x", "y", "z", "s", "t", "sdg", "tdg"], W.depolarizing_pauli(0.03, 1)),
         W.rule(["u3", "h"], W.amplitude_damping_kraus(0.04)),
         W.rule(["cx", "cz", "swap", "unitary"], W.depolarizing_pauli(0.06, 2))],
        readout=(0.02, 0.03))


@pytest.mark.parametrize("n,mode", [(10, "batch"), (10, "branch"), (11, "batch"), (12, "branch"),
                                    (12, "batch")])
def test_resident_groups_match_oracle(n, mode):
    circ = W.random_small(n, 120, seed=40 + n, n_mid=4, p_cond=0.3)
    noise = _noise()
    shots = 256
    say(f"case resident groups n={n} mode={mode} c128")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=17, engine=2)
    assert got["stats"]["tile_qubits"] == n and got["stats"]["groups"] > 0
    exp = oracle_memory(circ, noise, shots, seed=17)
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("n", [10, 12])
def test_resident_groups_layered_c1_shape(n):
    # the 10-qubit workload shape: U3 layers with CX pairings (the closing
    # CX of a group is applied by where its results are stored)
    circ = W.random_layered(n, 12, seed=n)
    noise = W.depol_model()
    shots = 500
    say(f"case resident layered n={n} c128")
    got = gpu_run(circ, noise, shots, dtype="c128", seed=5, engine=2)
    exp = oracle_memory(circ, noise, shots, seed=5)
    assert mismatches(got["memory"], exp) == 0


def test_resident_groups_dense_ops():
    circ = W.random_dense(11, 30, seed=8, n_mid=2)
    noise = _noise()
    say("case resident dense ops n=11 c128 batch")
    got = gpu_run(circ, noise, 200, dtype="c128", seed=23, engine=2)
    exp = oracle_memory(circ, noise, 200, seed=23)
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("n,dtype", [(10, "c128"), (13, "c64")])
def test_resident_groups_state(n, dtype):
    circ = W.random_layered(n, 6, seed=3 + n)
    noise = W.depol_model(p1=0.05, p2=0.1)
    say(f"case resident state dump n={n} {dtype}")
    got = gpu_run(circ, noise, 4, dtype=dtype, seed=9, dump_shot=2, engine=2)
    # the state kept is the one before the final measurement
    n_exp = len(dm.expand(circ, noise))
    _, exp = oracle.run(circ, noise, [2], seed=9, stop_at=n_exp - 1, want_state=True)
    tol = 1e-12 if dtype == "c128" else 2e-5
    assert np.max(np.abs(got["state"] - exp)) < tol


def test_resident_groups_complex64_agree():
    circ = W.random_layered(13, 15, seed=21)
    noise = W.workload("c3_20q")["noise"]
    shots = 2000
    say("case resident groups n=13 c64 against c128")
    a = gpu_run(circ, noise, shots, dtype="c64", seed=4, engine=2)["memory"]
    b = gpu_run(circ, noise, shots, dtype="c128", seed=4, engine=2)["memory"]
    assert np.mean(a == b) >= 0.99
