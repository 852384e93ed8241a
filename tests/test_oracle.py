"""Pins of the FP64 oracle against facts fixed outside it: published Philox
known answers, closed forms, special cases, exact brute force on small
circuits (two independent methods) and deterministic consequences of the
shared (seed, shot, op) draws. CPU only."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import dm
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def setup_module(_):
    oracle.build(force=False)


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_uniform_is_53bit_from_first_two_words():
    x = oracle.philox4x32_10([5, 0, 7, 0], [3, 0])
    u = oracle.uniform(3, 5, 7, 0)
    assert u == ((x[0] >> 5) * 2 ** 26 + (x[1] >> 6)) / 2.0 ** 53
    hi = oracle.philox4x32_10([0, 1, 2, 9], [0xFFFFFFFF, 0x1])
    assert oracle.uniform((1 << 32) | 0xFFFFFFFF, 1 << 32, 2, 9) == \
        ((hi[0] >> 5) * 2 ** 26 + (hi[1] >> 6)) / 2.0 ** 53


def test_uniform_statistics():
    us = np.array([oracle.uniform(11, s, 3, 0) for s in range(20000)])
    assert us.min() >= 0.0 and us.max() < 1.0
    assert abs(us.mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(us))
    assert abs(us.var() - 1 / 12) < 0.005
    # different d / r fields give uncorrelated streams
    vs = np.array([oracle.uniform(11, s, 3, 1) for s in range(20000)])
    assert abs(np.corrcoef(us, vs)[0, 1]) < 0.03


# --------------------------------------------------------------------------
# Gates: special cases, inverse round trip, agreement with an independent
# dense-matrix application
# --------------------------------------------------------------------------

def _state(circ, noise=None, shot=0, seed=0, stop_at=-1):
    _, psi = oracle.run(circ, noise, [shot], seed=seed, stop_at=stop_at,
                        want_state=True)
    return psi


def test_u3_special_cases():
    x = {"n_qubits": 1, "n_clbits": 0,
         "ops": [{"kind": "u3", "qubits": [0], "params": [math.pi, 0, math.pi]}]}
    psi = _state(x)
    assert abs(psi[0]) < 1e-15 and abs(psi[1] - 1) < 1e-15
    h = {"n_qubits": 1, "n_clbits": 0,
         "ops": [{"kind": "u3", "qubits": [0], "params": [math.pi / 2, 0, math.pi]}]}
    psi = _state(h)
    assert np.allclose(psi, [1 / math.sqrt(2), 1 / math.sqrt(2)], atol=1e-15)
    # U3(0, 0, lambda) is the phase gate diag(1, e^{i lambda}) on |+>
    p = {"n_qubits": 1, "n_clbits": 0,
         "ops": [{"kind": "h", "qubits": [0]},
                 {"kind": "u3", "qubits": [0], "params": [0, 0, 0.3]}]}
    psi = _state(p)
    assert np.allclose(psi, np.array([1, np.exp(0.3j)]) / math.sqrt(2), atol=1e-15)


def test_round_trip_returns_to_zero_state():
    circ = W.random_small(5, 60, seed=3, kinds=["u3", "h", "s", "t", "cx", "cz",
                                                 "swap"], measure_all=False)
    inv = []
    for op in reversed(circ["ops"]):
        k = op["kind"]
        if k == "u3":
            th, ph, la = op["params"]
            inv.append({"kind": "u3", "qubits": op["qubits"], "params": [-th, -la, -ph]})
        elif k in ("s", "t"):
            inv.append({"kind": k + "dg", "qubits": op["qubits"]})
        else:
            inv.append(op)
    full = dict(circ, ops=circ["ops"] + inv)
    psi = _state(full)
    assert abs(psi[0] - 1) < 1e-13
    assert np.max(np.abs(psi[1:])) < 1e-13


def test_gates_match_independent_dense_application():
    for seed in range(6):
        circ = W.random_small(4, 40, seed=seed, measure_all=False)
        psi = _state(circ)
        ref = np.zeros(16, dtype=complex)
        ref[0] = 1
        for op in circ["ops"]:
            ref = dm.embed(dm.gate_matrix(op), op["qubits"], 4) @ ref
        assert np.max(np.abs(psi - ref)) < 1e-13
        assert abs(np.vdot(psi, psi).real - 1) < 1e-13


# --------------------------------------------------------------------------
# Deterministic consequences of the shared draws
# --------------------------------------------------------------------------

def test_bell_outcome_follows_draw():
    circ = {"n_qubits": 2, "n_clbits": 2,
            "ops": [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 1]},
                    {"kind": "measure", "qubits": [0, 1], "clbits": [0, 1]}]}
    mem = oracle.run(circ, None, 4000, seed=9)
    assert set(np.unique(mem)) <= {0, 3}
    for s in range(4000):
        u = oracle.uniform(9, s, 2, 0)
        assert mem[s] == (0 if u < 0.5 else 3)


def test_ghz_counts():
    n = 5
    ops = [{"kind": "h", "qubits": [0]}] + \
        [{"kind": "cx", "qubits": [i, i + 1]} for i in range(n - 1)] + \
        [{"kind": "measure", "qubits": list(range(n)), "clbits": list(range(n))}]
    circ = {"n_qubits": n, "n_clbits": n, "ops": ops}
    mem = oracle.run(circ, None, 3000, seed=1)
    zeros = sum(1 for s in range(3000) if oracle.uniform(1, s, n, 0) < 0.5)
    assert int(np.sum(mem == 0)) == zeros
    assert int(np.sum(mem == 2 ** n - 1)) == 3000 - zeros


def test_table1_bitflip_follows_cumulative_threshold():
    # Table I: 1% bit flip, ID below 0.99, X from 0.99 to 1.00
    noise = W.noise_model([W.rule(["id"], W.pauli_table([0.99, 0.01], ["I", "X"]))])
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "id", "qubits": [0]},
                    {"kind": "measure", "qubits": [0], "clbits": [0]}]}
    mem = oracle.run(circ, noise, 20000, seed=4)
    for s in range(20000):
        assert mem[s] == (1 if oracle.uniform(4, s, 1, 0) >= 0.99 else 0)
    assert abs(mem.mean() - 0.01) < 4 * math.sqrt(0.01 * 0.99 / 20000)


def test_kraus_choice_follows_running_sum():
    g = 0.3
    noise = W.noise_model([W.rule(["h"], W.amplitude_damping_kraus(g))])
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "h", "qubits": [0]},
                    {"kind": "measure", "qubits": [0], "clbits": [0]}]}
    mem = oracle.run(circ, noise, 5000, seed=2)
    for s in range(5000):
        uk = oracle.uniform(2, s, 1, 0)
        um = oracle.uniform(2, s, 2, 0)
        if uk >= 1 - g / 2:          # K1 taken: |+> decays to |0>
            exp = 0
        else:                        # K0: (|0> + sqrt(1-g)|1>) / sqrt(2-g)
            exp = 0 if um < 1 / (2 - g) else 1
        assert mem[s] == exp, s


def test_decision_margin_closed_forms():
    # margin = distance from u*N to the nearest running-sum boundary of the
    # chosen candidate, over N. Bell measure: boundary 1/2, margin |u - 1/2|.
    # Amplitude damping on |+>: boundary p0 = 1 - g/2; the following measure
    # of the damped state has boundary 1/(2 - g) (K0) or none (K1: |0>, the
    # first outcome is certain and its upper boundary C_0 = N sits at the
    # top of the range). A circuit without Kraus or measure choices: +inf.
    bell = {"n_qubits": 2, "n_clbits": 2,
            "ops": [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 1]},
                    {"kind": "measure", "qubits": [0, 1], "clbits": [0, 1]}]}
    _, marg = oracle.run(bell, None, 500, seed=9, want_margins=True)
    for s in range(500):
        u = oracle.uniform(9, s, 2, 0)
        assert marg[s] == pytest.approx(abs(u - 0.5), abs=1e-15), s
    g = 0.3
    noise = W.noise_model([W.rule(["h"], W.amplitude_damping_kraus(g))])
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "h", "qubits": [0]},
                    {"kind": "measure", "qubits": [0], "clbits": [0]}]}
    _, marg = oracle.run(circ, noise, 500, seed=2, want_margins=True)
    for s in range(500):
        uk = oracle.uniform(2, s, 1, 0)
        um = oracle.uniform(2, s, 2, 0)
        mk = abs(uk - (1 - g / 2))
        if uk >= 1 - g / 2:          # K1: |0>, measure margin 1 - um (boundary C_0 = N)
            exp = min(mk, 1 - um)
        else:
            exp = min(mk, abs(um - 1 / (2 - g)))
        assert marg[s] == pytest.approx(exp, abs=1e-14), s
    free = {"n_qubits": 2, "n_clbits": 0, "ops": [{"kind": "h", "qubits": [0]}]}
    _, marg = oracle.run(free, W.depol_model(0.5, 0.5, gates1=("h",)), 4, seed=1,
                         want_margins=True)
    assert np.all(np.isinf(marg))


def test_readout_flip_draw():
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "measure", "qubits": [0], "clbits": [0]}]}
    noise = W.noise_model([], readout=(0.1, 0.0))
    mem = oracle.run(circ, noise, 5000, seed=8)
    for s in range(5000):
        assert mem[s] == (1 if oracle.uniform(8, s, 0, 1) < 0.1 else 0)


def test_reset_then_measure_is_zero():
    circ = {"n_qubits": 2, "n_clbits": 4,
            "ops": [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 1]},
                    {"kind": "measure_reset", "qubits": [0, 1], "clbits": [0, 1]},
                    {"kind": "measure", "qubits": [0, 1], "clbits": [2, 3]}]}
    mem = oracle.run(circ, None, 2000, seed=5)
    assert np.all((mem >> 2) == 0)
    assert set(np.unique(mem & 3)) == {0, 3}
    circ2 = {"n_qubits": 1, "n_clbits": 1,
             "ops": [{"kind": "h", "qubits": [0]}, {"kind": "reset", "qubits": [0]},
                     {"kind": "measure", "qubits": [0], "clbits": [0]}]}
    assert np.all(oracle.run(circ2, None, 500, seed=5) == 0)


def test_state_stays_normalised_through_kraus_and_measure():
    # the norm is checked after every expanded op (a later measurement would
    # renormalise a wrongly scaled Kraus result)
    noise = W.noise_model([W.rule(["u3"], W.amplitude_damping_kraus(0.2)),
                           W.rule(["cx"], W.depolarizing_pauli(0.3, 2))])
    circ = W.random_layered(3, 3, seed=2, measure_all=False,
                            mid_measure=(2, (0, 2)))
    n_x = len(dm.expand(circ, noise))
    for shot in range(6):
        for stop in range(1, n_x + 1):
            psi = _state(circ, noise, shot=shot, stop_at=stop)
            assert abs(np.vdot(psi, psi).real - 1) < 1e-12, (shot, stop)


# --------------------------------------------------------------------------
# Closed forms, exact brute force (density matrix == trajectory tree) and
# sampled oracle counts against them
# --------------------------------------------------------------------------

def _sample_check(mem, dist, n_shots, sig=5.0):
    for key, p in dist.items():
        c = int(np.sum(mem == key))
        sd = math.sqrt(max(p * (1 - p), 1e-12) * n_shots)
        assert abs(c - p * n_shots) <= sig * sd + 1, (key, c, p * n_shots)
    keys = set(int(k) for k in np.unique(mem))
    assert keys <= set(k for k, p in dist.items() if p > 0)


def test_depolarizing_closed_form():
    p, k = 0.05, 7
    noise = W.noise_model([W.rule(["id"], W.depolarizing_pauli(p, 1))])
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "id", "qubits": [0]}] * k +
                   [{"kind": "measure", "qubits": [0], "clbits": [0]}]}
    exact = (1 - (1 - p) ** k) / 2
    d = dm.creg_distribution_dm(circ, noise)
    assert abs(d[1] - exact) < 1e-13
    t = dm.creg_distribution_tree(circ, noise)
    assert abs(t[1] - exact) < 1e-13
    mem = oracle.run(circ, noise, 40000, seed=3)
    _sample_check(mem, d, 40000)


def test_two_qubit_depolarizing_zz_closed_form():
    p, k = 0.04, 5
    noise = W.noise_model([W.rule(["id"], W.depolarizing_pauli(p, 2))])
    # Bell pair, then k identity "gates" on both qubits carrying depol2 noise
    # (a two-qubit 'id' is expressed as a swap applied twice)
    ops = [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 1]}]
    noise2 = W.noise_model([W.rule(["swap"], W.depolarizing_pauli(p, 2))])
    ops += [{"kind": "swap", "qubits": [0, 1]}] * (2 * k)
    ops += [{"kind": "measure", "qubits": [0, 1], "clbits": [0, 1]}]
    circ = {"n_qubits": 2, "n_clbits": 2, "ops": ops}
    d = dm.creg_distribution_dm(circ, noise2)
    zz = d.get(0, 0) + d.get(3, 0) - d.get(1, 0) - d.get(2, 0)
    assert abs(zz - (1 - p) ** (2 * k)) < 1e-12
    # the tree has 16 branches per noise site: check it on two sites
    short = dict(circ, ops=ops[:4] + ops[-1:])
    t = dm.creg_distribution_tree(short, noise2)
    ds = dm.creg_distribution_dm(short, noise2)
    zzt = t.get(0, 0) + t.get(3, 0) - t.get(1, 0) - t.get(2, 0)
    assert abs(zzt - (1 - p) ** 2) < 1e-12
    assert dm.tvd(ds, t) < 1e-12
    mem = oracle.run(circ, noise2, 40000, seed=6)
    _sample_check(mem, d, 40000)


def test_amplitude_damping_closed_form():
    g, k = 0.1, 6
    noise = W.noise_model([W.rule(["id"], W.amplitude_damping_kraus(g))])
    for prep, factor in (("x", 1.0), ("h", 0.5)):
        circ = {"n_qubits": 1, "n_clbits": 1,
                "ops": [{"kind": prep, "qubits": [0]}] +
                       [{"kind": "id", "qubits": [0]}] * k +
                       [{"kind": "measure", "qubits": [0], "clbits": [0]}]}
        d = dm.creg_distribution_dm(circ, noise)
        assert abs(d[1] - factor * (1 - g) ** k) < 1e-13
        t = dm.creg_distribution_tree(circ, noise)
        assert abs(t[1] - factor * (1 - g) ** k) < 1e-13
        mem = oracle.run(circ, noise, 40000, seed=12)
        _sample_check(mem, d, 40000)


def test_readout_closed_form():
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "x", "qubits": [0]},
                    {"kind": "measure", "qubits": [0], "clbits": [0]}]}
    noise = W.noise_model([], readout=(0.0, 0.07))
    d = dm.creg_distribution_dm(circ, noise)
    assert abs(d[0] - 0.07) < 1e-15
    mem = oracle.run(circ, noise, 20000, seed=1)
    _sample_check(mem, d, 20000)


def _random_noise(seed):
    rng = np.random.default_rng(seed)
    # a random CPTP single-qubit Kraus channel from a random isometry
    z = rng.normal(size=(6, 2)) + 1j * rng.normal(size=(6, 2))
    v, _ = np.linalg.qr(z)
    mats = [v[2 * i:2 * i + 2, :] for i in range(3)]
    return W.noise_model(
        [W.rule(["u3", "h"], W.depolarizing_pauli(0.2, 1)),
         W.rule(["u3"], W.amplitude_damping_kraus(0.25)),
         W.rule(["t", "s"], W.kraus_channel(mats)),
         W.rule(["cx", "cz"], W.depolarizing_pauli(0.15, 2))],
        readout=(0.03, 0.06))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_dm_equals_tree_and_oracle_samples(seed):
    rng = np.random.default_rng(100 + seed)
    n = 2 + seed % 2
    circ = W.random_small(n, 4, seed=seed, kinds=["u3", "h", "t", "s", "cx", "cz"],
                          n_mid=1)
    noise = _random_noise(seed)
    d = dm.creg_distribution_dm(circ, noise)
    t = dm.creg_distribution_tree(circ, noise)
    assert abs(sum(d.values()) - 1) < 1e-12
    assert dm.tvd(d, t) < 1e-12
    shots = 30000
    mem = oracle.run(circ, noise, shots, seed=int(rng.integers(1 << 30)))
    _sample_check(mem, d, shots)


def test_oracle_sample_mismatch_detects_wrong_channel_order():
    # Depolarizing-then-damping and damping-then-depolarizing are different
    # channels; the sampled check must tell them apart (guards the rule
    # order of the noise expansion).
    circ = {"n_qubits": 1, "n_clbits": 1,
            "ops": [{"kind": "x", "qubits": [0]}, {"kind": "id", "qubits": [0]},
                    {"kind": "measure", "qubits": [0], "clbits": [0]}]}
    a = W.noise_model([W.rule(["x", "id"], W.pauli_table([0.5, 0.5], ["I", "X"])),
                       W.rule(["x", "id"], W.amplitude_damping_kraus(0.9))])
    b = W.noise_model([W.rule(["x", "id"], W.amplitude_damping_kraus(0.9)),
                       W.rule(["x", "id"], W.pauli_table([0.5, 0.5], ["I", "X"]))])
    da = dm.creg_distribution_dm(circ, a)
    db = dm.creg_distribution_dm(circ, b)
    assert dm.tvd(da, db) > 0.1
    mem = oracle.run(circ, a, 20000, seed=0)
    _sample_check(mem, da, 20000)


@pytest.mark.parametrize("x", [0, 1, 6, 19])
def test_qft_workload_is_the_discrete_fourier_transform(x):
    # the decomposed textbook QFT (H, phase, CX, three-CX swaps) maps |x>
    # to sum_y exp(2 pi i x y / N) |y> / sqrt(N): numpy's FFT is the check
    n = 5
    circ = W.qft(n, prepare=x, measure_all=False)
    noise = W.noise_model([])
    psi = _state(circ, noise, stop_at=len(dm.expand(circ, noise)))
    N = 1 << n
    expect = np.fft.ifft(np.eye(N)[x]) * math.sqrt(N)   # exp(+2 pi i x y / N) / sqrt(N)
    assert np.max(np.abs(psi - expect)) < 1e-14


def test_depolarizing_kraus_form_equals_pauli_form():
    # the same channel given as a Kraus list (Sec. III-B) reaches the same
    # exact distribution, and the oracle's Kraus selection samples it
    p, k = 0.05, 7
    ops = [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 1]}]
    ops += [{"kind": "id", "qubits": [0]}] * k + [{"kind": "swap", "qubits": [0, 1]}] * 2
    ops += [{"kind": "measure", "qubits": [0, 1], "clbits": [0, 1]}]
    circ = {"n_qubits": 2, "n_clbits": 2, "ops": ops}
    rules_p = [W.rule(["id"], W.depolarizing_pauli(p, 1)), W.rule(["swap"], W.depolarizing_pauli(p, 2))]
    rules_k = [W.rule(["id"], W.depolarizing_kraus(p, 1)), W.rule(["swap"], W.depolarizing_kraus(p, 2))]
    dp = dm.creg_distribution_dm(circ, W.noise_model(rules_p))
    dk = dm.creg_distribution_dm(circ, W.noise_model(rules_k))
    for key in range(4):
        assert abs(dp.get(key, 0.0) - dk.get(key, 0.0)) < 1e-13
    # one qubit, closed form
    one = {"n_qubits": 1, "n_clbits": 1,
           "ops": [{"kind": "id", "qubits": [0]}] * k + [{"kind": "measure", "qubits": [0], "clbits": [0]}]}
    nk = W.noise_model([W.rule(["id"], W.depolarizing_kraus(p, 1))])
    d1 = dm.creg_distribution_dm(one, nk)
    assert abs(d1[1] - (1 - (1 - p) ** k) / 2) < 1e-13
    mem = oracle.run(one, nk, 40000, seed=9)
    _sample_check(mem, d1, 40000)
    mem2 = oracle.run(circ, W.noise_model(rules_k), 20000, seed=4)
    _sample_check(mem2, dk, 20000)


def test_feed_forward_conditional_closed_form():
    # H, measure q0 -> c0, X on q1 only if c0 == 1, measure q1 -> c1:
    # the register is 00 or 11, each with probability 1/2 exactly, and with
    # readout error the conditional follows the recorded (flipped) bit
    ops = [{"kind": "h", "qubits": [0]},
           {"kind": "measure", "qubits": [0], "clbits": [0]},
           {"kind": "x", "qubits": [1], "cond": [1, 1]},
           {"kind": "measure", "qubits": [1], "clbits": [1]}]
    circ = {"n_qubits": 2, "n_clbits": 2, "ops": ops}
    d = dm.creg_distribution_dm(circ, None)
    assert abs(d[0] - 0.5) < 1e-14 and abs(d[3] - 0.5) < 1e-14
    assert all(v < 1e-15 for k, v in d.items() if k not in (0, 3))
    ro = (0.1, 0.2)
    dr = dm.creg_distribution_dm(circ, W.noise_model([], readout=ro))
    # c0 recorded 1 with prob (1/2)(p01) + (1/2)(1-p10); then q1 = 1 and c1 reads it
    pc0 = 0.5 * ro[0] + 0.5 * (1 - ro[1])
    assert abs(dr.get(3, 0) - pc0 * (1 - ro[1])) < 1e-14
    assert abs(dr.get(1, 0) - pc0 * ro[1]) < 1e-14
    assert abs(dr.get(2, 0) - (1 - pc0) * ro[0]) < 1e-14
    mem = oracle.run(circ, None, 20000, seed=2)
    assert set(np.unique(mem).tolist()) <= {0, 3}
    _sample_check(mem, d, 20000)


def test_branch_op_sets_bit_from_register():
    # Bell pair measured into c0 c1; the branch op writes c2 = (c0c1 == 11)
    ops = [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 1]},
           {"kind": "measure", "qubits": [0, 1], "clbits": [0, 1]},
           {"kind": "bfunc", "clbits": [2], "mask": 3, "value": 3},
           {"kind": "x", "qubits": [0], "cond": [4, 4]},
           {"kind": "measure", "qubits": [0], "clbits": [3]}]
    circ = {"n_qubits": 2, "n_clbits": 4, "ops": ops}
    d = dm.creg_distribution_dm(circ, None)
    # 00 -> c2=0, q0 stays 0; 11 -> c2=1, X flips q0 back to 0
    assert abs(d[0b0000] - 0.5) < 1e-14 and abs(d[0b0111] - 0.5) < 1e-14
    t = dm.creg_distribution_tree(circ, None)
    assert dm.tvd(d, t) < 1e-14
    mem = oracle.run(circ, None, 4000, seed=5)
    assert set(np.unique(mem).tolist()) <= {0b0000, 0b0111}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_conditionals_dm_equals_tree_and_oracle_samples(seed):
    n = 2
    circ = W.random_small(n, 5, seed=40 + seed, kinds=["u3", "h", "t", "s", "cx", "cz"],
                          n_mid=2, p_cond=0.7)
    assert any(op.get("cond") for op in circ["ops"])
    noise = _random_noise(seed)
    d = dm.creg_distribution_dm(circ, noise)
    t = dm.creg_distribution_tree(circ, noise)
    assert abs(sum(d.values()) - 1) < 1e-12
    assert dm.tvd(d, t) < 1e-12
    shots = 30000
    mem = oracle.run(circ, noise, shots, seed=17 + seed)
    _sample_check(mem, d, shots)


def test_multi_qubit_channels_dm_equals_tree_and_oracle():
    # dense 3-qubit unitaries followed by a random 3-qubit Kraus channel (4
    # matrices, not diagonal) and a random 3-qubit Pauli channel (64
    # terms): the exact register distribution by density matrices equals
    # the trajectory-tree enumeration, and oracle samples follow it
    rng = np.random.default_rng(5)
    ops = [{"kind": "h", "qubits": [0]}, {"kind": "cx", "qubits": [0, 3]}]
    for qs in ([0, 1, 2], [3, 1, 0]):
        ops.append({"kind": "unitary", "qubits": qs,
                    "matrix": W.haar_unitary(8, rng).tolist()})
    ops.append({"kind": "measure", "qubits": [0, 1, 2, 3], "clbits": [0, 1, 2, 3]})
    circ = {"n_qubits": 4, "n_clbits": 4, "ops": ops}
    noise = W.noise_model([W.rule(["unitary"], W.random_kraus(3, 4, seed=1)),
                           W.rule(["unitary"], W.random_pauli_channel(3, seed=2, p_noise=0.4))],
                          readout=(0.01, 0.02))
    d = dm.creg_distribution_dm(circ, noise)
    t = dm.creg_distribution_tree(circ, noise)
    assert abs(sum(d.values()) - 1) < 1e-12
    assert dm.tvd(d, t) < 1e-12
    mem = oracle.run(circ, noise, 30000, seed=3)
    _sample_check(mem, d, 30000)


@pytest.mark.parametrize("w", [3, 4, 5])
def test_dense_unitary_round_trip(w):
    # U then U^dagger on w qubits returns |0..0> up to rounding
    rng = np.random.default_rng(w)
    u = W.haar_unitary(1 << w, rng)
    qs = [int(x) for x in rng.choice(6, w, replace=False)]
    circ = {"n_qubits": 6, "n_clbits": 0,
            "ops": [{"kind": "h", "qubits": [q]} for q in range(6)] +
                   [{"kind": "unitary", "qubits": qs, "matrix": u.tolist()},
                    {"kind": "unitary", "qubits": qs, "matrix": u.conj().T.tolist()}] +
                   [{"kind": "h", "qubits": [q]} for q in range(6)]}
    _, psi = oracle.run(circ, None, [0], want_state=True)
    assert abs(psi[0] - 1) < 1e-13 and np.max(np.abs(psi[1:])) < 1e-13
