"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never loads it and
shares no code with it.

Two independent checkers of the multi-shot noisy state-vector method of
Doi, Horii and Wood (arXiv 2308.03399):

* ``run``       -- the plain per-shot FP64 trajectory simulator in
                   ``traj.c`` (C, OpenMP over shots).
* ``dm``        -- exact classical-register distributions for <= 5 qubits
                   by density-matrix evolution and by enumeration of the
                   trajectory tree (``dm.py``, NumPy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Iterable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

KIND = {"id": 0, "x": 1, "y": 2, "z": 3, "h": 4, "s": 5, "sdg": 6, "t": 7,
        "tdg": 8, "u3": 9, "cx": 16, "cz": 17, "swap": 18, "unitary": 24,
        "measure": 32, "reset": 33, "measure_reset": 34, "bfunc": 40}
PAULI_CODE = {"I": 0, "X": 1, "Y": 2, "Z": 3}
MAXQ = 32


def build(force: bool = True) -> str:
    """Compile traj.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp,
                               os.path.join(_HERE, "traj.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run.argtypes = [
            ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, P, P, ctypes.c_int,
            P, P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint64, ctypes.c_long, P, P, ctypes.c_int, P,
            ctypes.c_int, P]
        L.oracle_uniform.restype = ctypes.c_double
        L.oracle_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        _lib = L
    return _lib


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return [int(v) for v in out]


def uniform(seed: int, shot: int, r: int, d: int = 0) -> float:
    return float(lib().oracle_uniform(seed, shot, r, d))


def _pack(circuit: Dict, noise: Optional[Dict]):
    ops = circuit["ops"]
    n_ops = len(ops)
    kind = np.zeros(n_ops, dtype=np.int32)
    nq = np.zeros(n_ops, dtype=np.int32)
    q = np.full(n_ops * MAXQ, -1, dtype=np.int32)
    c = np.full(n_ops * MAXQ, -1, dtype=np.int32)
    par = np.zeros(n_ops * 3, dtype=np.float64)
    mat_off = np.full(n_ops, -1, dtype=np.int64)
    cmask = np.zeros(n_ops, dtype=np.uint64)
    cval = np.zeros(n_ops, dtype=np.uint64)
    mats = []
    moff = 0
    for i, op in enumerate(ops):
        kind[i] = KIND[op["kind"]]
        qs = list(op.get("qubits", []))
        if op["kind"] == "bfunc":           # predicate of the branch op
            cmask[i], cval[i] = int(op["mask"]), int(op["value"])
        elif op.get("cond"):                # condition of a conditional op
            cmask[i], cval[i] = int(op["cond"][0]), int(op["cond"][1])
        nq[i] = len(qs)
        q[i * MAXQ:i * MAXQ + len(qs)] = qs
        cl = list(op.get("clbits", []))
        c[i * MAXQ:i * MAXQ + len(cl)] = cl
        p = list(op.get("params", []))
        par[i * 3:i * 3 + len(p)] = p
        if op["kind"] == "unitary":
            m = np.asarray(op["matrix"], dtype=np.complex128)
            flat = np.empty(m.size * 2)
            flat[0::2] = m.real.ravel()
            flat[1::2] = m.imag.ravel()
            mats.append(flat)
            mat_off[i] = moff
            moff += flat.size
    mats = np.concatenate(mats) if mats else np.zeros(1)

    rules = (noise or {}).get("rules", [])
    n_rules = len(rules)
    gmask = np.zeros(max(n_rules, 1), dtype=np.uint32)
    rtype = np.zeros(max(n_rules, 1), dtype=np.int32)
    rnq = np.zeros(max(n_rules, 1), dtype=np.int32)
    rnt = np.zeros(max(n_rules, 1), dtype=np.int32)
    roff = np.zeros(max(n_rules, 1), dtype=np.int64)
    probs, codes, kmats = [], [], []
    poff = koff = 0
    for r, ru in enumerate(rules):
        m = 0
        for g in ru["gates"]:
            m |= 1 << KIND[g]
        gmask[r] = m
        rnq[r] = ru["nq"]
        if ru["type"] == "pauli":
            rtype[r] = 0
            rnt[r] = len(ru["probs"])
            roff[r] = poff
            probs.extend(float(p) for p in ru["probs"])
            for s in ru["paulis"]:
                row = [PAULI_CODE[ch] for ch in s]
                codes.extend(row + [0] * (MAXQ - len(row)))
            poff += len(ru["probs"])
        else:
            rtype[r] = 1
            rnt[r] = len(ru["mats"])
            roff[r] = koff
            for mm in ru["mats"]:
                a = np.asarray(mm, dtype=np.complex128)
                flat = np.empty(a.size * 2)
                flat[0::2] = a.real.ravel()
                flat[1::2] = a.imag.ravel()
                kmats.append(flat)
                koff += flat.size
    probs = np.asarray(probs if probs else [0.0], dtype=np.float64)
    codes = np.asarray(codes if codes else [0], dtype=np.int32)
    kmats = np.concatenate(kmats) if kmats else np.zeros(1)
    ro = (noise or {}).get("readout", [0.0, 0.0])
    return dict(kind=kind, nq=nq, q=q, c=c, par=par, cmask=cmask, cval=cval, mat_off=mat_off,
                mats=mats, n_rules=n_rules, gmask=gmask, rtype=rtype,
                rnq=rnq, rnt=rnt, roff=roff, probs=probs, codes=codes,
                kmats=kmats, ro01=float(ro[0]), ro10=float(ro[1]))


def run(circuit: Dict, noise: Optional[Dict], shots, seed: int = 0,
        n_threads: Optional[int] = None, stop_at: int = -1,
        want_state: bool = False, want_margins: bool = False):
    """Per-shot classical registers ("memory") for the given shot ids.

    ``shots``: an int (ids 0..shots-1) or an iterable of shot ids.
    With ``want_state`` only the first id is simulated and its state after
    ``stop_at`` expanded ops (all if negative) is returned as well.
    With ``want_margins`` the smallest relative decision margin of each shot
    (``traj.c`` header: distance of u*N to the nearest running-sum boundary
    of its Kraus and measure choices, over N; +inf without such a choice) is
    returned after the memory.
    """
    if isinstance(shots, (int, np.integer)):
        ids = np.arange(int(shots), dtype=np.int64)
    else:
        ids = np.asarray(list(shots), dtype=np.int64)
    if want_state:
        ids = ids[:1]
    a = _pack(circuit, noise)
    n = int(circuit["n_qubits"])
    mem = np.zeros(max(len(ids), 1), dtype=np.uint64)
    state = np.zeros(2 << n, dtype=np.float64) if want_state else None
    if n_threads is None:
        n_threads = len(os.sched_getaffinity(0))
    margins = np.zeros(max(len(ids), 1), dtype=np.float64)
    n_x = lib().oracle_run(
        n, len(circuit["ops"]), a["kind"].ctypes.data, a["nq"].ctypes.data,
        a["q"].ctypes.data, a["c"].ctypes.data, a["par"].ctypes.data,
        a["cmask"].ctypes.data, a["cval"].ctypes.data, a["mat_off"].ctypes.data, a["mats"].ctypes.data, a["n_rules"],
        a["gmask"].ctypes.data, a["rtype"].ctypes.data, a["rnq"].ctypes.data,
        a["rnt"].ctypes.data, a["roff"].ctypes.data, a["probs"].ctypes.data,
        a["codes"].ctypes.data, a["kmats"].ctypes.data, a["ro01"], a["ro10"],
        int(seed), len(ids), ids.ctypes.data, mem.ctypes.data, int(stop_at),
        state.ctypes.data if want_state else None, int(n_threads),
        margins.ctypes.data)
    if n_x < 0:
        raise ValueError("oracle rejected the circuit")
    mem = mem[:len(ids)]
    out = [mem]
    if want_state:
        out.append(state.view(np.complex128))
    if want_margins:
        out.append(margins[:len(ids)])
    return out[0] if len(out) == 1 else tuple(out)


def counts(memory: Iterable[int]) -> Dict[int, int]:
    out: Dict[int, int] = {}
    for m in memory:
        out[int(m)] = out.get(int(m), 0) + 1
    return out
