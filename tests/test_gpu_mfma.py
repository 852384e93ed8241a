"""complex64 fused one-qubit micro-ops on the matrix cores (option mfma):
a 2x2 complex matrix on an amplitude pair is a real 4x4 matrix, applied by
four accumulating v_mfma_f32_4x4x1f32 per pair. The kept state must equal
the FP64 oracle's amplitudes to complex64 rounding, and the per-shot
registers the oracle's (up to a near-tie), on streamed tiles with one or
two register sets and on LDS-resident states, in batch and branch mode.
The automatic choice takes the matrix cores for complex64; option mfma=1
keeps the vector ALU."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import gpu_run, mismatches, oracle_memory, say
from test_gpu_parity import _noise_full, len_expanded

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,tile", [(15, 13), (15, 12), (16, 14), (11, 0), (12, 0)])
def test_matrix_core_state_dump_matches_oracle(n, tile):
    circ = W.random_small(n, 120, seed=60 + n, measure_all=True)
    noise = _noise_full(p1=0.3, p2=0.3, gamma=0.3)
    _, psi = oracle.run(circ, noise, [2], seed=1,
                        stop_at=len_expanded(circ, noise) - 1, want_state=True)
    opts = {"tile_qubits": tile} if tile else {}
    for mf in (1, 2):
        say(f"case mfma={mf} dump n={n} tile={tile}")
        got = gpu_run(circ, noise, 4, dtype="c64", seed=1, dump_shot=2, mfma=mf, **opts)
        assert got["stats"]["mfma"] == (1 if mf == 2 else 0)
        assert np.max(np.abs(got["state"] - psi)) < 5e-5


@pytest.mark.parametrize("mode", ["batch", "branch"])
def test_matrix_core_registers_match_oracle(mode):
    n = 15
    circ = W.random_layered(n, 5, seed=23, mid_measure=(2, (0, n - 1)))
    noise = _noise_full(p1=0.02, p2=0.04, gamma=0.03)
    shots = 128
    say(f"case mfma registers mode={mode}")
    got = gpu_run(circ, noise, shots, dtype="c64", mode=mode, seed=7, tile_qubits=13, mfma=2)
    assert got["stats"]["mfma"] == 1
    exp = oracle_memory(circ, noise, shots, seed=7)
    assert mismatches(got["memory"], exp) <= 1


def test_automatic_choice_is_the_matrix_cores_for_complex64():
    # measured faster on both the 20-qubit workload (2.6 one-qubit gates per
    # register group) and the 26-qubit one (5.6): complex64 takes the
    # matrix cores unless option mfma=1 asks for the vector ALU
    dense = W.random_layered(16, 12, seed=0, two_qubit="cz")
    say("case mfma automatic, U3+CZ layers")
    got = gpu_run(dense, W.depol_model(gates2=("cz",)), 8, dtype="c64", seed=0, tile_qubits=13)
    assert got["stats"]["mfma"] == 1
    sparse = W.workload("c3_20q")
    say("case mfma automatic, 20-qubit workload circuit")
    got = gpu_run(sparse["circuit"], sparse["noise"], 4, dtype="c64", seed=0)
    assert got["stats"]["mfma"] == 1
    got = gpu_run(sparse["circuit"], sparse["noise"], 4, dtype="c64", seed=0, mfma=1)
    assert got["stats"]["mfma"] == 0
    got = gpu_run(dense, W.depol_model(gates2=("cz",)), 8, dtype="c128", seed=0, tile_qubits=12)
    assert got["stats"]["mfma"] == 0  # complex128 always on the vector ALU
