"""GPU parity: per-shot classical registers of the HIP path equal the FP64
oracle's, shot by shot, through the C ABI. FP64 (c128) storage must match
exactly; c64 storage (FP64 decisions) is held to agreement-rate and TVD
bounds."""
import math

import numpy as np
import pytest

import oracle
import paper_2308_03399_amd as S
import workloads as W
from gpu_util import gpu_run, mismatches, oracle_memory, say, tvd_counts

pytestmark = pytest.mark.gpu


def _noise_full(p1=0.02, p2=0.05, gamma=0.03, ro=(0.02, 0.03)):
    return W.noise_model(
        [W.rule(["u3", "h", "x", "y", "z", "s", "t", "sdg", "tdg"],
                W.depolarizing_pauli(p1, 1)),
         W.rule(["u3", "h"], W.amplitude_damping_kraus(gamma)),
         W.rule(["cx", "cz", "swap", "unitary"], W.depolarizing_pauli(p2, 2))],
        readout=ro)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_small_random_circuits_c128_exact(n):
    circ = W.random_small(n, 40, seed=n, n_mid=3 if n > 1 else 0)
    noise = _noise_full()
    shots = 600
    say(f"case small n={n} shots={shots} c128 batch")
    got = gpu_run(circ, noise, shots, dtype="c128", seed=7)
    exp = oracle_memory(circ, noise, shots, seed=7)
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("mode,n,tile", [("batch", 6, 0), ("branch", 6, 0), ("plain", 6, 0),
                                         ("batch", 14, 12), ("branch", 14, 12)])
def test_decision_margins_match_oracle(mode, n, tile):
    # measurement-only decisions (Pauli noise, mid-circuit measures, final
    # sampling): both sides take the same choices from the same running
    # sums, so the smallest margin of every shot agrees to rounding
    circ = W.random_small(n, 60, seed=20 + n, n_mid=4)
    noise = W.noise_model([W.rule(["u3", "h"], W.depolarizing_pauli(0.05, 1)),
                           W.rule(["cx", "cz", "swap", "unitary"], W.depolarizing_pauli(0.05, 2))])
    shots = 200 if mode != "plain" else 24
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case margins mode={mode} n={n} tile={tile}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=13, want_margins=True, **opts)
    exp, marg = oracle.run(circ, noise, shots, seed=13, want_margins=True)
    assert mismatches(got["memory"], exp) == 0
    assert np.allclose(got["margins"], marg, rtol=1e-9, atol=1e-13)
    assert got["stats"]["near_ties"] == int(np.sum(got["margins"] < 1e-9))


@pytest.mark.parametrize("mode,n,tile", [("batch", 5, 0), ("branch", 14, 12)])
def test_one_qubit_rule_on_mixed_width_unitaries(mode, n, tile):
    # a one-qubit Kraus channel on the "unitary" kind attaches after the
    # one-qubit unitaries only, as the oracle expands it
    rng = np.random.default_rng(4)

    def haar(d):
        z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        q, r = np.linalg.qr(z)
        return (q * (np.diag(r) / abs(np.diag(r)))).tolist()

    ops = []
    for _ in range(12):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        ops.append({"kind": "unitary", "qubits": [a], "matrix": haar(2)})
        ops.append({"kind": "unitary", "qubits": [a, b], "matrix": haar(4)})
    ops.append({"kind": "measure", "qubits": list(range(n)), "clbits": list(range(n))})
    circ = {"n_qubits": n, "n_clbits": n, "ops": ops}
    noise = W.noise_model([W.rule(["unitary"], W.amplitude_damping_kraus(0.2))])
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case mixed-width unitary rule mode={mode} n={n}")
    got = gpu_run(circ, noise, 128, dtype="c128", mode=mode, seed=5, **opts)
    assert mismatches(got["memory"], oracle_memory(circ, noise, 128, seed=5)) == 0


def _dense_noise():
    # rules attach by width: a random 3-qubit Kraus channel (4 matrices)
    # and a random 3-qubit Pauli channel (64 terms) after the 3-qubit
    # unitaries, a random 4-qubit Kraus channel (3 matrices) after the
    # 4-qubit ones, a random 5-qubit Pauli channel (1024 terms) after the
    # 5-qubit ones
    return W.noise_model(
        [W.rule(["u3"], W.amplitude_damping_kraus(0.05)),
         W.rule(["unitary"], W.random_kraus(3, 4, seed=1)),
         W.rule(["unitary"], W.random_pauli_channel(3, seed=2, p_noise=0.3)),
         W.rule(["unitary"], W.random_kraus(4, 3, seed=3)),
         W.rule(["unitary"], W.random_pauli_channel(5, seed=4, p_noise=0.3)),
         W.rule(["cx"], W.depolarizing_pauli(0.05, 2))],
        readout=(0.01, 0.02))


@pytest.mark.parametrize("mode,n,tile", [("batch", 6, 0), ("branch", 6, 0), ("plain", 7, 0),
                                         ("batch", 15, 12), ("branch", 15, 12),
                                         ("batch", 15, 13), ("branch", 16, 13)])
def test_dense_multi_qubit_ops_match_oracle(mode, n, tile):
    # dense unitaries on 3, 4 and 5 qubits with multi-qubit Kraus and Pauli
    # channels, mid-circuit measures; complex128, resident (n <= tile) and
    # streamed tiles (dense ops as LDS sweeps, 3-qubit Pauli strings fused
    # into register groups, the 5-qubit ones as LDS sweeps when they exceed
    # the group width); branch mode splits 1024-term Pauli draws by rank
    circ = W.random_dense(n, 30, seed=30 + n + tile, n_mid=2)
    noise = _dense_noise()
    shots = 128 if mode != "plain" else 16
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case dense multi-qubit ops mode={mode} n={n} tile={tile}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=9, **opts)
    exp = oracle_memory(circ, noise, shots, seed=9)
    assert mismatches(got["memory"], exp) == 0
    if mode == "branch":
        assert got["stats"]["branches"] >= 1


def test_dense_multi_qubit_ops_complex64():
    circ = W.random_dense(15, 30, seed=61, n_mid=2)
    noise = _dense_noise()
    say("case dense multi-qubit ops c64 n=15 tile 13")
    got = gpu_run(circ, noise, 256, dtype="c64", seed=9, tile_qubits=13)
    exp = oracle_memory(circ, noise, 256, seed=9)
    assert mismatches(got["memory"], exp) <= 3


def test_op_wider_than_the_tile_is_refused():
    # a 5-qubit unitary on high qubits with qubits 0..3 needs 9 tile qubits
    import paper_2308_03399_amd as S
    rng = np.random.default_rng(0)
    circ = {"n_qubits": 12, "n_clbits": 0,
            "ops": [{"kind": "unitary", "qubits": [7, 8, 9, 10, 11],
                     "matrix": W.haar_unitary(32, rng).tolist()}]}
    sim = S.Simulator(12, 4, dtype="c64", tile_qubits=8)
    try:
        with pytest.raises(S.SvError) as e:
            sim.run(circ, None, seed=0)
        assert e.value.status == 5  # SV_EUNSUPPORTED
    finally:
        sim.close()


def test_c1_workload_exact():
    w = W.workload("c1_10q")
    say("case c1 10q x 20 layers, 1000 shots, c128 batch")
    got = gpu_run(w["circuit"], w["noise"], w["shots"], dtype="c128", seed=w["seed"])
    exp = oracle_memory(w["circuit"], w["noise"], w["shots"], seed=w["seed"])
    assert mismatches(got["memory"], exp) == 0
    cnt = got["counts"]
    assert sum(cnt.values()) == w["shots"]
    ek, ec = np.unique(exp, return_counts=True)
    assert cnt == {int(k): int(c) for k, c in zip(ek, ec)}


@pytest.mark.parametrize("tile", [6, 8])
def test_streamed_tiles_exact(tile):
    # state larger than the tile: ops run in tile sweeps through HBM
    n = 11
    circ = W.random_layered(n, 6, seed=3, mid_measure=(3, (0, 5)))
    noise = _noise_full(p1=0.03, p2=0.06, gamma=0.05)
    shots = 200
    say(f"case streamed n={n} tile={tile} shots={shots} c128 batch")
    got = gpu_run(circ, noise, shots, dtype="c128", seed=11, tile_qubits=tile)
    exp = oracle_memory(circ, noise, shots, seed=11)
    assert got["stats"]["tile_qubits"] == tile
    assert got["stats"]["passes"] > 0
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("n,tile", [(6, 0), (11, 8)])
def test_dump_state_matches_oracle(n, tile):
    circ = W.random_layered(n, 4, seed=5)
    noise = _noise_full(p1=0.2, p2=0.2, gamma=0.2)
    shot = 13
    say(f"case dump n={n} tile={tile}")
    for dtype, tol in (("c128", 1e-12), ("c64", 2e-5)):
        opts = {"tile_qubits": tile} if tile else {}
        got = gpu_run(circ, noise, 20, dtype=dtype, seed=2, dump_shot=shot, **opts)
        _, psi = oracle.run(circ, noise, [shot], seed=2,
                            stop_at=len_expanded(circ, noise) - 1, want_state=True)
        assert np.max(np.abs(got["state"] - psi)) < tol, dtype


def len_expanded(circ, noise):
    from oracle import dm
    return len(dm.expand(circ, noise))


@pytest.mark.parametrize("n,tile", [(5, 0), (11, 7)])
def test_branch_mode_equals_batch_and_oracle(n, tile):
    circ = W.random_layered(n, 5, seed=9, mid_measure=(2, (1,)))
    noise = _noise_full(p1=0.01, p2=0.03, gamma=0.02)
    shots = 400
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case branch n={n} tile={tile} shots={shots}")
    br = gpu_run(circ, noise, shots, dtype="c128", mode="branch", seed=4, **opts)
    exp = oracle_memory(circ, noise, shots, seed=4)
    assert mismatches(br["memory"], exp) == 0
    st = br["stats"]
    assert st["branches"] >= 1
    # fewer states than shots were simulated
    assert st["branches"] < shots


def test_branch_mode_waiting_list_restarts():
    n = 9
    circ = W.random_layered(n, 4, seed=2)
    noise = _noise_full(p1=0.05, p2=0.1, gamma=0.05)
    shots = 300
    say("case branch waiting list (2 slots)")
    br = gpu_run(circ, noise, shots, dtype="c128", mode="branch", seed=8,
                 tile_qubits=6, slots=2, workers=4)
    exp = oracle_memory(circ, noise, shots, seed=8)
    assert br["stats"]["restarts"] >= 1
    assert mismatches(br["memory"], exp) == 0


def test_c64_agreement_and_tvd():
    w = W.workload("c1_10q")
    shots = 1000
    say("case c64 c1 agreement")
    got = gpu_run(w["circuit"], w["noise"], shots, dtype="c64", seed=0)
    exp = oracle_memory(w["circuit"], w["noise"], shots, seed=0)
    agree = 1 - mismatches(got["memory"], exp) / shots
    say(f"c64 agreement {agree:.5f}")
    assert agree >= 0.995
    assert tvd_counts(got["memory"], exp) <= 5e-3


# ---------------------------------------------------------------------------
# Register-group engine (tiles of 2^k with k = 8 + log2(amplitudes/thread))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tile,n,pipe", [("c64", 14, 16, 0), ("c64", 13, 15, 0),
                                               ("c128", 13, 15, 0), ("c128", 12, 14, 0),
                                               ("c64", 13, 15, 1), ("c64", 13, 17, 1),
                                               ("c128", 12, 14, 1), ("c64", 12, 14, 0),
                                               ("c64", 12, 14, 1)])
def test_group_engine_matches_oracle(dtype, tile, n, pipe):
    circ = W.random_layered(n, 5, seed=21, mid_measure=(2, (0, n - 1)))
    noise = _noise_full(p1=0.02, p2=0.04, gamma=0.03)
    shots = 64
    say(f"case groups dtype={dtype} tile={tile} n={n} pipeline={pipe} shots={shots}")
    got = gpu_run(circ, noise, shots, dtype=dtype, seed=5, tile_qubits=tile, pipeline=pipe)
    exp = oracle_memory(circ, noise, shots, seed=5)
    st = got["stats"]
    assert st["tile_qubits"] == tile
    assert st["tile_buffers"] == 1 + pipe
    bad = mismatches(got["memory"], exp)
    if dtype == "c128":
        assert bad == 0
    else:
        assert bad <= 1


@pytest.mark.parametrize("dtype,tile,pipe", [("c64", 14, 0), ("c128", 13, 0),
                                             ("c64", 13, 1), ("c128", 12, 1)])
def test_group_engine_state_dump(dtype, tile, pipe):
    n = 15
    circ = W.random_small(n, 120, seed=4, measure_all=True)
    noise = _noise_full(p1=0.3, p2=0.3, gamma=0.3)
    say(f"case groups dump dtype={dtype} tile={tile} pipeline={pipe}")
    got = gpu_run(circ, noise, 4, dtype=dtype, seed=1, dump_shot=2, tile_qubits=tile,
                  pipeline=pipe)
    assert got["stats"]["tile_buffers"] == 1 + pipe
    _, psi = oracle.run(circ, noise, [2], seed=1,
                        stop_at=len_expanded(circ, noise) - 1, want_state=True)
    tol = 1e-11 if dtype == "c128" else 5e-5
    assert np.max(np.abs(got["state"] - psi)) < tol


@pytest.mark.parametrize("pipe", [0, 1])
def test_group_engine_branch_mode(pipe):
    n = 15
    circ = W.random_layered(n, 4, seed=8, mid_measure=(2, (3,)))
    noise = _noise_full(p1=0.01, p2=0.02, gamma=0.02)
    shots = 256
    say(f"case groups branch mode pipeline={pipe}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode="branch", seed=6, pipeline=pipe)
    exp = oracle_memory(circ, noise, shots, seed=6)
    assert mismatches(got["memory"], exp) == 0
    assert got["stats"]["branches"] > 0


def test_shot_offset_waves_equal_one_job():
    # a job run as two waves (shot_offset) equals the same shots in one run
    circ = W.random_layered(15, 4, seed=2)
    noise = _noise_full(p1=0.02, p2=0.04, gamma=0.03)
    say("case shot_offset waves")
    exp = oracle_memory(circ, noise, 300, seed=9)
    a = gpu_run(circ, noise, 120, dtype="c128", seed=9)
    b = gpu_run(circ, noise, 180, dtype="c128", seed=9, shot_offset=120)
    assert mismatches(a["memory"], exp[:120]) == 0
    assert mismatches(b["memory"], exp[120:]) == 0


# ---------------------------------------------------------------------------
# Plain per-shot form (one kernel per op over the whole state)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 9, 13])
def test_plain_mode_matches_oracle(n):
    circ = W.random_small(n, 60, seed=30 + n, n_mid=2)
    noise = _noise_full(p1=0.05, p2=0.08, gamma=0.05)
    shots = 40
    say(f"case plain n={n}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode="plain", seed=3)
    exp = oracle_memory(circ, noise, shots, seed=3)
    assert mismatches(got["memory"], exp) == 0


def test_plain_mode_c1_first_shots():
    w = W.workload("c1_10q")
    say("case plain c1 (100 shots)")
    got = gpu_run(w["circuit"], w["noise"], 100, dtype="c128", mode="plain", seed=0)
    exp = oracle_memory(w["circuit"], w["noise"], 100, seed=0)
    assert mismatches(got["memory"], exp) == 0


def test_largest_state_offsets_beyond_32_bits():
    # 29 qubits in complex128 is an 8 GiB state: tile copies address it with
    # offsets past 2^32 bytes
    n = 29
    ops = [{"kind": "u3", "qubits": [q], "params": [0.3 + 0.1 * q, 0.2, 0.1]} for q in (0, 13, 27, 28)]
    ops += [{"kind": "cx", "qubits": [28, 2]}, {"kind": "cx", "qubits": [14, 28]},
            {"kind": "u3", "qubits": [28], "params": [1.1, 0.4, -0.3]},
            {"kind": "measure", "qubits": [28, 27, 2, 0], "clbits": [0, 1, 2, 3]}]
    circ = {"n_qubits": n, "ops": ops}
    noise = W.noise_model([W.rule(["u3"], W.depolarizing_pauli(0.2, 1))])
    say("case largest state n=29 c128")
    got = gpu_run(circ, noise, 2, dtype="c128", seed=3, dump_shot=1)
    exp = oracle_memory(circ, noise, 2, seed=3)
    assert mismatches(got["memory"], exp) == 0
    # the last op is not a terminal measure-all, so the dump follows it
    _, psi = oracle.run(circ, noise, [1], seed=3, stop_at=len_expanded(circ, noise),
                        want_state=True)
    assert np.max(np.abs(got["state"] - psi)) < 1e-12


# ---------------------------------------------------------------------------
# The paper's QFT workload (Sec. V): H, phase and CX with depolarizing noise
# as a Pauli channel or as the equivalent Kraus list (16 matrices for CX)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form,mode,n,tile", [("pauli", "batch", 9, 0), ("kraus", "batch", 9, 0),
                                              ("kraus", "branch", 9, 0), ("kraus", "batch", 14, 12),
                                              ("pauli", "branch", 14, 12), ("kraus", "plain", 9, 0)])
def test_qft_workload_matches_oracle(form, mode, n, tile):
    circ = W.qft(n, prepare=5)
    noise = W.qft_noise(0.05, form)
    shots = 96 if mode != "plain" else 24
    say(f"case qft form={form} mode={mode} n={n} tile={tile}")
    opts = {"tile_qubits": tile} if tile else {}
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=11, **opts)
    exp = oracle_memory(circ, noise, shots, seed=11)
    assert mismatches(got["memory"], exp) == 0


# ---------------------------------------------------------------------------
# Conditional operations and branch ops on the classical register (Sec. IV-A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,mode,tile,dtype", [(3, "batch", 0, "c128"), (6, "branch", 0, "c128"),
                                               (14, "batch", 12, "c128"), (14, "branch", 12, "c128"),
                                               (14, "batch", 13, "c64")])
def test_conditional_circuits_match_oracle(n, mode, tile, dtype):
    circ = W.random_small(n, 60, seed=31 + n, n_mid=5, p_cond=0.5)
    assert sum(1 for op in circ["ops"] if op.get("cond")) >= 3
    noise = _noise_full(p1=0.05, p2=0.08, gamma=0.05)   # readout flips make cregs differ
    shots = 128
    say(f"case conditional n={n} mode={mode} tile={tile} dtype={dtype}")
    opts = {"tile_qubits": tile} if tile else {}
    got = gpu_run(circ, noise, shots, dtype=dtype, mode=mode, seed=13, **opts)
    exp = oracle_memory(circ, noise, shots, seed=13)
    bad = mismatches(got["memory"], exp)
    assert bad == 0 if dtype == "c128" else bad <= 1


def test_feed_forward_in_branch_mode_splits_by_register():
    # H, measure q0 -> c0, X on q1 iff c0 == 1, branch op c2 = (c0 == 1),
    # Z on q0 iff c2 == 1, final measure of both
    ops = [{"kind": "h", "qubits": [0]},
           {"kind": "measure", "qubits": [0], "clbits": [0]},
           {"kind": "x", "qubits": [1], "cond": [1, 1]},
           {"kind": "bfunc", "clbits": [2], "mask": 1, "value": 1},
           {"kind": "z", "qubits": [0], "cond": [4, 4]},
           {"kind": "measure", "qubits": [0, 1], "clbits": [0, 1]}]
    circ = {"n_qubits": 2, "n_clbits": 3, "ops": ops}
    noise = W.noise_model([], readout=(0.1, 0.1))
    shots = 512
    say("case feed-forward branch")
    got = gpu_run(circ, noise, shots, dtype="c128", mode="branch", seed=3)
    exp = oracle_memory(circ, noise, shots, seed=3)
    assert mismatches(got["memory"], exp) == 0


def test_plain_mode_refuses_conditional_circuits():
    circ = {"n_qubits": 2, "n_clbits": 1,
            "ops": [{"kind": "measure", "qubits": [0], "clbits": [0]},
                    {"kind": "x", "qubits": [1], "cond": [1, 1]}]}
    with pytest.raises(S.SvError) as e:
        gpu_run(circ, None, 4, dtype="c128", mode="plain")
    assert e.value.status == 5


# ---------------------------------------------------------------------------
# Full-size workloads, in the launch shapes the benchmark uses; the oracle
# checks sampled shot ids one by one
# ---------------------------------------------------------------------------
def test_c2_full_size_sampled_shots():
    w = W.workload("c2_16q")
    shots = w["shots"]
    say(f"case c2 16q x 40 layers with mid-circuit measure+reset, {shots} shots c128")
    got = gpu_run(w["circuit"], w["noise"], shots, dtype="c128", seed=w["seed"])
    ids = list(range(128)) + list(range(shots - 128, shots))
    exp = oracle.run(w["circuit"], w["noise"], ids, seed=w["seed"])
    assert mismatches(np.asarray(got["memory"])[ids], exp) == 0
    say("case c2 c64")
    got64 = gpu_run(w["circuit"], w["noise"], shots, dtype="c64", seed=w["seed"])
    agree = float(np.mean(np.asarray(got64["memory"])[ids] == exp))
    assert agree >= 0.99
    assert tvd_counts(got64["memory"], got["memory"]) <= 0.03   # sampling noise at 10k shots


def test_c3_full_size_sampled_shots():
    # one benchmark wave: 10,000 shots of the 20-qubit, 60-layer workload in
    # complex64 with the default launch shape; oracle on its first and last ids
    w = W.workload("c3_20q")
    shots = 10_000
    say(f"case c3 20q x 60 layers, {shots} shots c64 (one benchmark wave)")
    got = gpu_run(w["circuit"], w["noise"], shots, dtype="c64", seed=w["seed"])
    ids = list(range(8)) + list(range(shots - 8, shots))
    exp = oracle.run(w["circuit"], w["noise"], ids, seed=w["seed"])
    agree = int(np.sum(np.asarray(got["memory"])[ids] == exp))
    assert agree >= len(ids) - 1
    say("case c3 c128, 512 shots")
    got128 = gpu_run(w["circuit"], w["noise"], 512, dtype="c128", seed=w["seed"])
    ids128 = list(range(4)) + list(range(508, 512))
    exp128 = oracle.run(w["circuit"], w["noise"], ids128, seed=w["seed"])
    assert mismatches(np.asarray(got128["memory"])[ids128], exp128) == 0


def test_c3_full_size_branch_mode():
    # the benchmark's branch wave: 10,000 shots sharing states until their
    # draws split them (one slot per shot). In complex64 it agrees with the
    # batch wave within complex64 rounding (a shared state can be scaled
    # differently before a reduction), and in complex128 it is the oracle's
    w = W.workload("c3_20q")
    shots = 10_000
    say(f"case c3 branch mode, {shots} shots c64, against batch")
    br = gpu_run(w["circuit"], w["noise"], shots, dtype="c64", mode="branch", seed=w["seed"])
    ba = gpu_run(w["circuit"], w["noise"], shots, dtype="c64", seed=w["seed"])
    st = br["stats"]
    assert st["restarts"] == 0 and st["branches"] >= 1
    agree = float(np.mean(br["memory"] == ba["memory"]))
    say(f"branch/batch agreement {agree:.5f}, passes/shot {st['passes'] / shots:.2f}")
    assert agree >= 0.995
    say("case c3 branch mode c128, 256 shots")
    got = gpu_run(w["circuit"], w["noise"], 256, dtype="c128", mode="branch", seed=w["seed"])
    ids = list(range(4)) + list(range(252, 256))
    exp = oracle.run(w["circuit"], w["noise"], ids, seed=w["seed"])
    assert mismatches(np.asarray(got["memory"])[ids], exp) == 0


# ---------------------------------------------------------------------------
# Parameter sweeps: circuits differing only in U3 angles, one launch
# ---------------------------------------------------------------------------
def _with_angles(circ, angles):
    ops, u = [], 0
    for op in circ["ops"]:
        if op["kind"] == "u3":
            op = dict(op, params=[float(x) for x in angles[u]])
            u += 1
        ops.append(op)
    return dict(circ, ops=ops)


@pytest.mark.parametrize("n,dtype,tile", [(8, "c128", 0), (15, "c128", 12), (15, "c64", 13)])
def test_parameter_sweep_matches_oracle_per_set(n, dtype, tile):
    circ = W.random_layered(n, 4, seed=17, mid_measure=(2, (0,)))
    noise = _noise_full(p1=0.03, p2=0.05, gamma=0.04)
    n_u3 = sum(1 for op in circ["ops"] if op["kind"] == "u3")
    n_sets, per = 4, 24
    params = np.random.default_rng(5).uniform(0, 2 * math.pi, (n_sets, n_u3, 3))
    say(f"case sweep n={n} dtype={dtype} tile={tile} sets={n_sets}")
    opts = {"tile_qubits": tile} if tile else {}
    sim = S.Simulator(n, n_sets * per, dtype=dtype, spin_limit_ms=60000, **opts)
    try:
        sim.run_sweep(circ, noise, params, seed=8)
        mem = sim.memory()
    finally:
        sim.close()
    bad = 0
    for s in range(n_sets):
        ids = list(range(s * per, (s + 1) * per))
        exp = oracle.run(_with_angles(circ, params[s]), noise, ids, seed=8)
        bad += mismatches(np.asarray(mem)[ids], exp)
    assert bad == 0 if dtype == "c128" else bad <= 2


@pytest.mark.parametrize("n,tile", [(6, 0), (14, 12)])
def test_parameter_sweep_with_conditional_ops(n, tile):
    # swept U3 angles together with conditional gates and branch ops: each
    # set's shots are the oracle's shots of the circuit with that set's angles
    circ = W.random_small(n, 60, seed=23, n_mid=3, p_cond=0.4)
    noise = _noise_full(p1=0.03, p2=0.05, gamma=0.04)
    n_u3 = sum(1 for op in circ["ops"] if op["kind"] == "u3")
    assert n_u3 > 0 and any(op.get("cond") for op in circ["ops"])
    n_sets, per = 3, 20
    params = np.random.default_rng(9).uniform(0, 2 * math.pi, (n_sets, n_u3, 3))
    say(f"case sweep with conditions n={n} tile={tile}")
    opts = {"tile_qubits": tile} if tile else {}
    sim = S.Simulator(n, n_sets * per, dtype="c128", spin_limit_ms=60000, **opts)
    try:
        sim.run_sweep(circ, noise, params, seed=4)
        mem = sim.memory()
    finally:
        sim.close()
    for s in range(n_sets):
        ids = list(range(s * per, (s + 1) * per))
        exp = oracle.run(_with_angles(circ, params[s]), noise, ids, seed=4)
        assert mismatches(np.asarray(mem)[ids], exp) == 0


def _ladder(n, reps, seed, u3=True):
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(reps):
        if u3:
            for q in range(n):
                ops.append({"kind": "u3", "qubits": [q],
                            "params": [float(x) for x in rng.uniform(0, 2 * math.pi, 3)]})
        for q in range(n - 1):
            ops.append({"kind": "cx", "qubits": [q, q + 1]})
    ops.append({"kind": "measure", "qubits": list(range(n)), "clbits": list(range(n))})
    return {"n_qubits": n, "n_clbits": n, "ops": ops}


@pytest.mark.parametrize("n,tile,u3,mode", [(12, 0, False, "batch"), (12, 0, False, "branch"),
                                            (12, 0, True, "batch"), (12, 0, True, "branch"),
                                            (10, 0, False, "batch"), (14, 12, True, "batch")])
def test_passes_cut_at_group_and_matrix_room(n, tile, u3, mode):
    # A 12-qubit complex128 state on the register-group engine plans passes
    # of up to 512 ops. A CX ladder then gives 92 register groups in one
    # pass (a pass holds 64), and U3 layers 135 fused one-qubit matrices
    # (a pass holds 96): the fusion cuts the pass there and the next pass
    # continues. Registers must equal the oracle's
    circ = _ladder(n, 30, seed=n + tile, u3=u3)
    noise = W.depol_model(p1=0.02, p2=0.05)
    shots = 48
    opts = {"tile_qubits": tile} if tile else {}
    if n == 12:
        opts["engine"] = 2
    say(f"case pass cuts n={n} tile={tile} u3={u3} mode={mode}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=8, **opts)
    assert mismatches(got["memory"], oracle_memory(circ, noise, shots, seed=8)) == 0


@pytest.mark.parametrize("n,mode", [(12, "batch"), (12, "branch"), (14, "batch")])
def test_pass_cut_inside_one_register_group(n, mode):
    # 300 CX gates on one pair form a single register group per pass; with
    # strong two-qubit Pauli noise each CX flushes drawn factors, so a shot's
    # pass needs more micro-ops than a pass holds (384) and is cut inside
    # its first group
    ops = [{"kind": "u3", "qubits": [q], "params": [0.3 * (q + 1), 0.2, 0.1]} for q in range(n)]
    ops += [{"kind": "cx", "qubits": [0, 1]}] * 300
    ops.append({"kind": "measure", "qubits": list(range(n)), "clbits": list(range(n))})
    circ = {"n_qubits": n, "n_clbits": n, "ops": ops}
    noise = W.depol_model(p1=0.05, p2=0.3)
    shots = 32
    opts = {"engine": 2} if n == 12 else {"tile_qubits": 13}
    say(f"case cut inside one group n={n} mode={mode}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=9, **opts)
    assert mismatches(got["memory"], oracle_memory(circ, noise, shots, seed=9)) == 0
