"""Edge cases on the GPU, through the C ABI: empty and measurement-free
circuits, one shot, shot counts that leave ragged waves, noise and readout
that happen with probability 0 or 1, outcomes of probability 0, the
resident / streamed size boundary and the largest state (30 qubits).
Expected values are closed forms, or the FP64 oracle's per-shot registers."""
import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_run, mismatches, oracle_memory, say

pytestmark = pytest.mark.gpu


def _op(kind, qubits, params=None, clbits=None):
    o = {"kind": kind, "qubits": list(qubits)}
    if params is not None:
        o["params"] = list(params)
    if clbits is not None:
        o["clbits"] = list(clbits)
    return o


def _measure_all(n):
    return _op("measure", range(n), clbits=range(n))


def _noise_full():
    return W.noise_model(
        [W.rule(["u3", "h", "x"], W.depolarizing_pauli(0.03, 1)),
         W.rule(["u3", "h", "x"], W.amplitude_damping_kraus(0.04)),
         W.rule(["cx", "cz"], W.depolarizing_pauli(0.06, 2))],
        readout=(0.02, 0.03))


@pytest.mark.parametrize("mode", ["batch", "branch", "plain"])
@pytest.mark.parametrize("n", [3, 16])
def test_empty_circuit(mode, n):
    circ = {"n_qubits": n, "n_clbits": n, "ops": []}
    shots = 37
    say(f"case empty circuit n={n} {mode}")
    dump = 0 if mode == "batch" else None
    got = gpu_run(circ, _noise_full(), shots, dtype="c64", mode=mode, dump_shot=dump)
    assert np.all(got["memory"] == 0)
    assert got["counts"] == {0: shots}
    if dump is not None:
        st = got["state"]
        assert st[0] == 1 and np.count_nonzero(st) == 1


@pytest.mark.parametrize("n,tile", [(5, 0), (14, 12)])
def test_circuit_without_measurement(n, tile):
    circ = W.random_layered(n, 3, seed=4, measure_all=False)
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case no measurement n={n}")
    got = gpu_run(circ, _noise_full(), 50, dtype="c128", seed=2, **opts)
    assert np.all(got["memory"] == 0)
    assert got["counts"] == {0: 50}


@pytest.mark.parametrize("mode", ["batch", "branch"])
def test_single_shot_streamed(mode):
    circ = W.random_layered(15, 4, seed=8, mid_measure=(2, (0, 3)))
    noise = _noise_full()
    say(f"case one shot n=15 {mode}")
    got = gpu_run(circ, noise, 1, dtype="c128", mode=mode, seed=11, shot_offset=77)
    exp = oracle_memory(circ, noise, 78, seed=11)[77:]
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("mode,shots,opts", [
    ("batch", 23, {"workers": 7}),
    ("batch", 513, {}),
    ("branch", 37, {"workers": 5, "slots": 3}),
])
def test_ragged_shot_counts(mode, shots, opts):
    circ = W.random_layered(14, 3, seed=6, mid_measure=(1, (2,)))
    noise = _noise_full()
    say(f"case ragged {mode} shots={shots} {opts}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=5, **opts)
    exp = oracle_memory(circ, noise, shots, seed=5)
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["batch", "branch"])
@pytest.mark.parametrize("n", [5, 14])
def test_certain_pauli_noise(n, mode, dtype):
    # identity gates, each followed by an X with probability 1: every qubit
    # ends in |1>, so every shot reads all ones
    circ = {"n_qubits": n, "n_clbits": n,
            "ops": [_op("u3", [q], (0.0, 0.0, 0.0)) for q in range(n)] + [_measure_all(n)]}
    noise = W.noise_model([W.rule(["u3"], W.pauli_table([0, 1, 0, 0], ["I", "X", "Y", "Z"]))])
    say(f"case certain X noise n={n} {mode} {dtype}")
    got = gpu_run(circ, noise, 40, dtype=dtype, mode=mode, seed=1)
    assert np.all(got["memory"] == (1 << n) - 1)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_certain_readout_flips(dtype):
    # |q0 q2 = 1> measured, every recorded bit flipped: 0b0101 -> 0b1010
    n = 4
    circ = {"n_qubits": n, "n_clbits": n,
            "ops": [_op("x", [0]), _op("x", [2]), _measure_all(n)]}
    noise = W.noise_model([], readout=(1.0, 1.0))
    say(f"case certain readout flips {dtype}")
    got = gpu_run(circ, noise, 30, dtype=dtype, seed=3)
    assert np.all(got["memory"] == 0b1010)


@pytest.mark.parametrize("mode", ["batch", "branch"])
@pytest.mark.parametrize("n,tile", [(3, 0), (15, 12)])
def test_zero_probability_outcomes(n, tile, mode):
    # measuring and resetting a qubit in |0> always reads 0, and the reset
    # qubit reads 0 again; after X a qubit reads 1 with certainty
    ops = []
    for _ in range(3):
        ops.append(_op("h", [1]))
        ops.append(_op("h", [1]))  # with damping between, qubit 1 is left mixed
        ops.append(_op("measure_reset", [0, 1], clbits=[n, n + 1]))
    ops.append(_op("x", [n - 1]))
    ops.append(_measure_all(n))
    circ = {"n_qubits": n, "n_clbits": n + 2, "ops": ops}
    noise = W.noise_model([W.rule(["h"], W.amplitude_damping_kraus(0.9))])
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case zero-probability outcomes n={n} {mode}")
    got = gpu_run(circ, noise, 60, dtype="c128", mode=mode, seed=9, **opts)
    # qubit 1 after H, damping, H is random: compare with the oracle
    exp = oracle_memory(circ, noise, 60, seed=9)
    assert mismatches(got["memory"], exp) == 0
    mem = got["memory"]
    one = np.uint64(1)
    # certain bits: the last qubit reads 1; qubit 0 (never touched) reads 0
    # mid-circuit; qubits 0 and 1 were reset, so the final measure reads 0
    assert np.all(((mem >> np.uint64(n - 1)) & one) == one)
    assert np.all(((mem >> np.uint64(n)) & one) == 0)
    assert np.all((mem & np.uint64(0b11)) == 0)


@pytest.mark.parametrize("dtype,n", [("c64", 13), ("c64", 14), ("c128", 12), ("c128", 13)])
def test_resident_streamed_boundary(dtype, n):
    circ = W.random_layered(n, 4, seed=12, mid_measure=(2, (1,)))
    noise = _noise_full()
    shots = 200
    say(f"case boundary {dtype} n={n}")
    got = gpu_run(circ, noise, shots, dtype=dtype, seed=4)
    exp = oracle_memory(circ, noise, shots, seed=4)
    bad = mismatches(got["memory"], exp)
    if dtype == "c128":
        assert bad == 0
    else:
        assert bad <= 2
    resident = got["stats"]["tile_qubits"] == n
    assert resident == (n <= (13 if dtype == "c64" else 12))


def test_largest_state_thirty_qubits():
    # 8 GiB complex64 state: H on q0, X on q29, CX(29 -> 1), measure all
    n = 30
    circ = {"n_qubits": n, "n_clbits": n,
            "ops": [_op("h", [0]), _op("x", [29]), _op("cx", [29, 1]), _measure_all(n)]}
    say("case 30 qubits, c64, 8 shots")
    got = gpu_run(circ, None, 8, dtype="c64", seed=2)
    base = (1 << 29) | (1 << 1)
    mem = got["memory"]
    assert set(int(x) for x in mem) <= {base, base | 1}


def test_device_wait_timeout_is_reported_and_the_handle_recovers():
    # failure handling forced from the host: a 1 ms bound on the work-queue
    # waits of branch mode, counted as elapsed time rather than time without
    # progress. Idle workgroups give up waiting while the root record runs
    # its unsplit prefix (every wave still exits normally), the run reports
    # SV_EDEVICE, and the same handle runs correctly once the progress
    # watchdog is restored
    import paper_2308_03399_amd as S
    circ = W.random_layered(16, 20, seed=41)
    noise = W.depol_model()
    shots = 64
    say("case forced device wait timeout (branch mode, 1 ms)")
    sim = S.Simulator(16, shots, dtype="c128", mode="branch", spin_limit_ms=1, spin_elapsed=1)
    try:
        with pytest.raises(S.SvError) as e:
            sim.run(circ, noise, seed=3)
        assert e.value.status == 3  # SV_EDEVICE
        assert "device executor failed" in str(e.value)
        S.sv_batch_set_option(sim.h, "spin_elapsed", 0)
        sim.run(circ, noise, seed=3)
        mem1 = sim.memory()
        S.sv_batch_set_option(sim.h, "spin_limit_ms", 60000)
        sim.run(circ, noise, seed=3)
        mem = sim.memory()
    finally:
        sim.close()
    exp = oracle_memory(circ, noise, shots, seed=3)
    assert mismatches(mem, exp) == 0
    # the progress watchdog at the same 1 ms bound: the waits outlast 1 ms
    # while the root record runs, but sweeps keep completing, so the run
    # succeeds
    assert mismatches(mem1, exp) == 0


@pytest.mark.parametrize("n,shots", [(6, 1000), (16, 3001)])
def test_counts_histogram_contract(n, shots):
    # sv_sample_counts: ascending keys with their counts, equal to the
    # histogram of the per-shot registers; a too-small capacity returns
    # SV_EINVAL with the required size written
    import ctypes
    import paper_2308_03399_amd as S
    circ = W.random_layered(n, 3, seed=51)
    noise = _noise_full()
    say(f"case counts contract n={n} shots={shots}")
    sim = S.Simulator(n, shots, dtype="c64")
    try:
        sim.run(circ, noise, seed=6)
        mem = sim.memory()
        keys, cnt = np.unique(mem, return_counts=True)
        L = S.lib()
        nu = ctypes.c_size_t(0)
        # size query with no output arrays
        st = L.sv_sample_counts(sim.h, None, None, 0, ctypes.byref(nu))
        assert st == (1 if len(keys) > 0 else 0) and nu.value == len(keys)
        # one slot short
        k = np.zeros(len(keys), np.uint64)
        c = np.zeros(len(keys), np.uint64)
        nu.value = 0
        st = L.sv_sample_counts(sim.h, k.ctypes.data, c.ctypes.data, len(keys) - 1,
                                ctypes.byref(nu))
        assert st == 1 and nu.value == len(keys)
        # exact capacity
        st = L.sv_sample_counts(sim.h, k.ctypes.data, c.ctypes.data, len(keys), ctypes.byref(nu))
        assert st == 0 and nu.value == len(keys)
    finally:
        sim.close()
    assert np.array_equal(k, keys) and np.array_equal(c, cnt.astype(np.uint64))
    assert int(c.sum()) == shots


@pytest.mark.parametrize("mode,n,tile", [("batch", 5, 0), ("batch", 14, 12), ("branch", 14, 12)])
def test_random_keying_with_64_bit_seed_and_shot_ids(mode, n, tile):
    # Philox counter (shot lo, shot hi, r, d) and key (seed lo, seed hi): a
    # 64-bit seed and shot ids that cross 2^32 reach both high words
    circ = W.random_layered(n, 3, seed=61, mid_measure=(1, (0,)))
    noise = _noise_full()
    seed = 0xDEADBEEFCAFEF00D
    base = (1 << 32) - 5
    shots = 10
    opts = {"tile_qubits": tile} if tile else {}
    say(f"case 64-bit keying {mode} n={n}")
    got = gpu_run(circ, noise, shots, dtype="c128", mode=mode, seed=seed, shot_offset=base, **opts)
    exp = oracle_memory(circ, noise, range(base, base + shots), seed=seed)
    assert mismatches(got["memory"], exp) == 0


@pytest.mark.parametrize("mode", ["batch", "branch"])
def test_plan_reuse_across_circuits_on_one_handle(mode):
    # a handle keeps the last circuit's pass plan while the circuit's
    # structure repeats; a different structure must plan afresh, and the
    # same structure with other angles must reuse the plan correctly
    import paper_2308_03399_amd as S
    n, shots = 15, 64
    noise = _noise_full()
    a = W.random_layered(n, 4, seed=31, mid_measure=(2, (1, 7)))
    b = W.random_small(n, 80, seed=32, n_mid=2)
    a2 = W.random_layered(n, 4, seed=31, mid_measure=(2, (1, 7)))
    for op in a2["ops"]:  # same structure, other angles
        if op["kind"] == "u3":
            op["params"] = [p + 0.25 for p in op["params"]]
    sim = S.Simulator(n, shots, dtype="c128", mode=mode, tile_qubits=13, spin_limit_ms=60000)
    try:
        for name, circ, seed in (("A", a, 4), ("B", b, 5), ("A", a, 6), ("A'", a2, 7)):
            say(f"case plan reuse mode={mode} circuit {name} seed {seed}")
            sim.run(circ, noise, seed=seed)
            got = sim.memory()
            assert mismatches(got, oracle_memory(circ, noise, shots, seed=seed)) == 0, name
    finally:
        sim.close()
