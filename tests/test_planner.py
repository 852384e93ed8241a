"""Host-side execution planner (no GPU): the device order is a permutation
of the expanded op list that keeps the order of ops sharing a qubit and the
relative order of state-dependent random ops (Kraus, measure, reset); every
pass fits its tile and every register group its register bits."""
import ctypes

import numpy as np
import pytest

import paper_2308_03399_amd as S
import workloads as W
from oracle import dm


def _plan(circ, noise, tile_q, reg_bits):
    L = S.lib()
    f = L.svb_debug_plan
    P = ctypes.c_void_p
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(S.sv_op),
                  ctypes.c_size_t, ctypes.POINTER(S.sv_noise_model), P, P, P, P, P,
                  ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                  ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    m = S.marshal(circ, noise)
    cap = 200_000
    order = np.zeros(cap, np.int32)
    opass = np.zeros(cap, np.int32)
    ogrp = np.zeros(cap, np.int32)
    pmask = np.zeros(cap, np.uint32)
    gw = np.zeros(cap, np.int32)
    n = ctypes.c_size_t()
    np_ = ctypes.c_size_t()
    ng = ctypes.c_size_t()
    st = f(circ["n_qubits"], tile_q, reg_bits, m["ops"], m["n_ops"], m["nm"],
           order.ctypes.data, opass.ctypes.data, ogrp.ctypes.data, pmask.ctypes.data,
           gw.ctypes.data, cap, ctypes.byref(n), ctypes.byref(np_), ctypes.byref(ng))
    assert st == 0, S.sv_last_error()
    return (order[:n.value], opass[:n.value], ogrp[:n.value], pmask[:np_.value],
            gw[:ng.value])


def _is_ordered_random(x):
    return (x["kind"] == "channel" and x["rule"]["type"] == "kraus") or \
        x["kind"] in ("measure", "reset", "measure_reset", "bfunc") or bool(x.get("cond"))


@pytest.mark.parametrize("case", ["c3", "c2", "small", "cond"])
@pytest.mark.parametrize("tile_q,reg_bits", [(13, 5), (14, 6), (12, 4), (8, 0)])
def test_plan_respects_dependencies(case, tile_q, reg_bits):
    if case == "c3":
        w = W.workload("c3_20q")
        circ = dict(w["circuit"], ops=w["circuit"]["ops"][:900] + w["circuit"]["ops"][-1:])
        noise = w["noise"]
    elif case == "c2":
        w = W.workload("c2_16q")
        circ, noise = w["circuit"], w["noise"]
    elif case == "cond":
        circ = W.random_small(16, 300, seed=6, n_mid=8, p_cond=0.3)
        noise = W.noise_model([W.rule(["u3", "h"], W.amplitude_damping_kraus(0.1)),
                               W.rule(["cx", "cz"], W.depolarizing_pauli(0.1, 2))])
    else:
        circ = W.random_small(16, 300, seed=5, n_mid=6)
        noise = W.noise_model([W.rule(["u3", "h"], W.amplitude_damping_kraus(0.1)),
                               W.rule(["cx", "cz"], W.depolarizing_pauli(0.1, 2))])
    xo = dm.expand(circ, noise)
    order, opass, ogrp, pmask, gw = _plan(circ, noise, tile_q, reg_bits)
    assert sorted(order.tolist()) == list(range(len(xo)))
    pos = np.empty(len(xo), np.int64)
    pos[order] = np.arange(len(xo))
    last_on_qubit = {}
    last_random = -1
    for j, x in enumerate(xo):
        for q in x.get("qubits", []):
            if q in last_on_qubit:
                assert pos[last_on_qubit[q]] < pos[j], ("qubit order", q, j)
            last_on_qubit[q] = j
        if _is_ordered_random(x):
            if last_random >= 0:
                assert pos[last_random] < pos[j], ("random order", j)
            last_random = j
    n = circ["n_qubits"]
    k = min(tile_q, n)
    for p, m in enumerate(pmask):
        assert bin(int(m)).count("1") == k
    for d, j in enumerate(order):
        qm = sum(1 << q for q in xo[j].get("qubits", []))
        if len(xo[j].get("qubits", [])) < n:  # the final measure-all has its own pass
            assert (qm & ~int(pmask[opass[d]])) == 0
        if reg_bits > 0 and n > tile_q:
            assert gw[ogrp[d]] <= reg_bits
    # passes and groups are contiguous in device order
    assert np.all(np.diff(opass) >= 0)
    assert np.all(np.diff(ogrp) >= 0)


def test_plan_reorders_to_fewer_passes_than_list_order():
    w = W.workload("c3_20q")
    order, opass, _, _, _ = _plan(w["circuit"], w["noise"], 13, 5)
    layers = 60
    assert opass.max() + 1 < 3 * layers  # list-order planning needs about 3 per layer


def test_tile_set_search_is_deterministic_and_packs_passes():
    # streamed states: each pass's tile set is the best of the greedy set,
    # seeded candidates and single-qubit exchanges. The plan must not depend
    # on anything but the circuit, and the search must reach the pass counts
    # it was measured at (the greedy planner alone made 135 static passes on
    # the 20-qubit circuit and 116 on the 26-qubit one, terminal pass included)
    for name, k, most in (("c3_20q", 13, 131), ("c4_26q", 13, 89)):
        w = W.workload(name)
        a = _plan(w["circuit"], w["noise"], k, k - 8)
        b = _plan(w["circuit"], w["noise"], k, k - 8)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert len(a[3]) <= most, (name, len(a[3]))


def test_rule_attaches_only_to_gates_of_its_width():
    # a one-qubit channel on the "unitary" kind: expanded after the 1-qubit
    # unitaries only, as the oracle expands it (the plan holds every
    # expanded op once)
    rng = np.random.default_rng(3)

    def haar(d):
        z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        q, r = np.linalg.qr(z)
        return q * (np.diag(r) / abs(np.diag(r)))

    ops = [{"kind": "unitary", "qubits": [0], "matrix": haar(2)},
           {"kind": "unitary", "qubits": [1, 2], "matrix": haar(4)},
           {"kind": "unitary", "qubits": [2], "matrix": haar(2)},
           {"kind": "measure", "qubits": [0, 1, 2], "clbits": [0, 1, 2]}]
    circ = {"n_qubits": 3, "n_clbits": 3, "ops": ops}
    noise = W.noise_model([W.rule(["unitary"], W.amplitude_damping_kraus(0.2))])
    order, _, _, _, _ = _plan(circ, noise, 3, 0)
    assert sorted(order.tolist()) == list(range(6))  # 4 ops + 2 channels
