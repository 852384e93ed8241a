"""Exact classical-register distributions for small circuits -- TEST
INFRASTRUCTURE ONLY (part of the oracle).

Two independent exact methods, used to pin the trajectory oracle:

* ``creg_distribution_dm``   -- density-matrix evolution that carries one
  (unnormalised) density matrix per classical-register value. Pauli and
  Kraus channels act as sum_j E_j rho E_j^dagger, a measurement splits rho
  by projector and readout confusion (the noise model of Sec. III-B of
  Doi, Horii and Wood, arXiv 2308.03399, in its density-matrix form, the
  comparison method named in Sec. II).
* ``creg_distribution_tree`` -- enumeration of every trajectory of the
  multi-shot method (Sec. III-B Pauli sampling and Kraus selection,
  Sec. IV-A measure/reset), weighted by its probability.

Both expand noise sites after every matching gate in rule order (the
all-qubit rule of the paper's noise-model example). Only for <= 5 qubits.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

_I2 = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)
_PAULI = {"I": _I2, "X": _X, "Y": _Y, "Z": _Z}
_GATES_2Q = ("cx", "cz", "swap")
_NON_GATES = ("measure", "reset", "measure_reset")


def gate_matrix(op: Dict) -> np.ndarray:
    """Matrix of a gate over its qubit list; bit t of the row/column index is
    the value of op['qubits'][t]."""
    k = op["kind"]
    if k == "u3":
        th, ph, la = op["params"]
        return np.array([[math.cos(th / 2), -np.exp(1j * la) * math.sin(th / 2)],
                         [np.exp(1j * ph) * math.sin(th / 2),
                          np.exp(1j * (ph + la)) * math.cos(th / 2)]])
    fixed = {"id": _I2, "x": _X, "y": _Y, "z": _Z,
             "h": np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2),
             "s": np.diag([1, 1j]), "sdg": np.diag([1, -1j]),
             "t": np.diag([1, np.exp(1j * math.pi / 4)]),
             "tdg": np.diag([1, np.exp(-1j * math.pi / 4)])}
    if k in fixed:
        return np.asarray(fixed[k], dtype=complex)
    if k == "cx":  # qubits [control, target]; index = c + 2 t
        m = np.zeros((4, 4), dtype=complex)
        for c in range(2):
            for t in range(2):
                m[c + 2 * (t ^ c), c + 2 * t] = 1
        return m
    if k == "cz":
        return np.diag([1, 1, 1, -1]).astype(complex)
    if k == "swap":
        m = np.zeros((4, 4), dtype=complex)
        for a in range(2):
            for b in range(2):
                m[b + 2 * a, a + 2 * b] = 1
        return m
    if k == "unitary":
        return np.asarray(op["matrix"], dtype=complex)
    raise KeyError(k)


def embed(m: np.ndarray, qubits: List[int], n: int) -> np.ndarray:
    """Full 2^n x 2^n operator of a k-qubit matrix acting on ``qubits``."""
    dim = 1 << n
    full = np.zeros((dim, dim), dtype=complex)
    mask = 0
    for q in qubits:
        mask |= 1 << q
    for i in range(dim):
        a = sum(((i >> q) & 1) << t for t, q in enumerate(qubits))
        for b in range(m.shape[1]):
            j = i & ~mask
            for t, q in enumerate(qubits):
                if (b >> t) & 1:
                    j |= 1 << q
            full[i, j] = m[a, b]
    return full


def _pauli_matrix(s: str) -> np.ndarray:
    # character t acts on qubit-list position t (bit t of the index)
    out = np.array([[1]], dtype=complex)
    for ch in s:
        out = np.kron(_PAULI[ch], out)
    return out


def expand(circuit: Dict, noise: Dict) -> List[Dict]:
    """Noise sites after every matching gate; a conditional gate's channels
    carry its condition."""
    rules = (noise or {}).get("rules", [])
    out = []
    for op in circuit["ops"]:
        out.append(op)
        if op["kind"] in _NON_GATES or op["kind"] == "bfunc":
            continue
        for ru in rules:
            if op["kind"] in ru["gates"] and ru["nq"] == len(op["qubits"]):
                out.append({"kind": "channel", "rule": ru, "cond": op.get("cond"),
                            "qubits": list(op["qubits"])})
    return out


def _holds(op: Dict, creg: int) -> bool:
    """Condition of an op (Sec. IV-A conditional gates): (creg & mask) == value."""
    cond = op.get("cond")
    return not cond or (creg & int(cond[0])) == int(cond[1])


def _bfunc(op: Dict, creg: int) -> int:
    """Branch op: its clbit becomes ((creg & mask) == value)."""
    bit = 1 if (creg & int(op["mask"])) == int(op["value"]) else 0
    cb = op["clbits"][0]
    return (creg & ~(1 << cb)) | (bit << cb)


def _channel_ops(ru: Dict) -> List[Tuple[float, np.ndarray]]:
    """(probability or None, matrix) list of a channel."""
    if ru["type"] == "pauli":
        return [(float(p), _pauli_matrix(s)) for p, s in
                zip(ru["probs"], ru["paulis"])]
    return [(None, np.asarray(m, dtype=complex)) for m in ru["mats"]]


def _confusion(bit: int, rec: int, ro) -> float:
    p01, p10 = ro
    if bit == 0:
        return p01 if rec == 1 else 1.0 - p01
    return p10 if rec == 0 else 1.0 - p10


def _set_bits(creg: int, clbits: List[int], pattern: int) -> int:
    for t, cb in enumerate(clbits):
        creg = (creg & ~(1 << cb)) | (((pattern >> t) & 1) << cb)
    return creg


def _projector(n: int, qubits: List[int], pattern: int) -> np.ndarray:
    d = np.zeros(1 << n)
    for i in range(1 << n):
        if all(((i >> q) & 1) == ((pattern >> t) & 1)
               for t, q in enumerate(qubits)):
            d[i] = 1.0
    return np.diag(d).astype(complex)


def _reset_op(n: int, qubits: List[int], pattern: int) -> np.ndarray:
    """X on each measured qubit whose outcome bit is 1."""
    m = np.eye(1 << n, dtype=complex)
    for t, q in enumerate(qubits):
        if (pattern >> t) & 1:
            m = embed(_X, [q], n) @ m
    return m


def creg_distribution_dm(circuit: Dict, noise: Dict) -> Dict[int, float]:
    n = circuit["n_qubits"]
    ro = (noise or {}).get("readout", [0.0, 0.0])
    rho0 = np.zeros((1 << n, 1 << n), dtype=complex)
    rho0[0, 0] = 1.0
    states = {0: rho0}
    for op in expand(circuit, noise):
        new: Dict[int, np.ndarray] = {}
        k = op["kind"]
        if k == "bfunc":
            for cr, rho in states.items():
                key = _bfunc(op, cr)
                new[key] = new.get(key, 0) + rho
            states = new
            continue
        # registers whose condition fails keep their state untouched
        skipped = {cr: rho for cr, rho in states.items() if not _holds(op, cr)}
        states = {cr: rho for cr, rho in states.items() if _holds(op, cr)}
        if k == "channel":
            mats = [(p, embed(m, op["qubits"], n)) for p, m in
                    _channel_ops(op["rule"])]
            for cr, rho in states.items():
                acc = np.zeros_like(rho)
                for p, E in mats:
                    w = 1.0 if p is None else p
                    acc += w * (E @ rho @ E.conj().T)
                new[cr] = acc
        elif k in _NON_GATES:
            qs = op["qubits"]
            m = len(qs)
            for cr, rho in states.items():
                for pat in range(1 << m):
                    P = _projector(n, qs, pat)
                    r = P @ rho @ P
                    if k != "measure":
                        R = _reset_op(n, qs, pat)
                        r = R @ r @ R.conj().T
                    if k == "reset":
                        new[cr] = new.get(cr, 0) + r
                        continue
                    for rec in range(1 << m):
                        w = 1.0
                        for t in range(m):
                            w *= _confusion((pat >> t) & 1, (rec >> t) & 1, ro)
                        if w == 0.0:
                            continue
                        key = _set_bits(cr, op["clbits"], rec)
                        new[key] = new.get(key, 0) + w * r
        else:
            U = embed(gate_matrix(op), op["qubits"], n)
            for cr, rho in states.items():
                new[cr] = U @ rho @ U.conj().T
        for cr, rho in skipped.items():
            new[cr] = new.get(cr, 0) + rho
        states = new
    return {cr: float(np.real(np.trace(rho))) for cr, rho in states.items()}


def creg_distribution_tree(circuit: Dict, noise: Dict,
                           prune: float = 0.0) -> Dict[int, float]:
    n = circuit["n_qubits"]
    ro = (noise or {}).get("readout", [0.0, 0.0])
    xops = expand(circuit, noise)
    full = {}
    for i, op in enumerate(xops):
        if op["kind"] == "bfunc":
            continue
        if op["kind"] == "channel":
            full[i] = [(p, embed(m, op["qubits"], n)) for p, m in
                       _channel_ops(op["rule"])]
        elif op["kind"] not in _NON_GATES:
            full[i] = embed(gate_matrix(op), op["qubits"], n)
        else:
            m = len(op["qubits"])
            full[i] = [(_projector(n, op["qubits"], pat),
                        _reset_op(n, op["qubits"], pat)) for pat in range(1 << m)]
    out: Dict[int, float] = {}

    def walk(i: int, psi: np.ndarray, w: float, creg: int):
        if w <= prune:
            return
        if i == len(xops):
            out[creg] = out.get(creg, 0.0) + w
            return
        op = xops[i]
        k = op["kind"]
        if k == "bfunc":
            walk(i + 1, psi, w, _bfunc(op, creg))
            return
        if not _holds(op, creg):
            walk(i + 1, psi, w, creg)
            return
        if k == "channel":
            for p, E in full[i]:
                phi = E @ psi
                q = float(np.vdot(phi, phi).real)
                if p is None:  # Kraus: branch weight is ||K psi||^2
                    if q > 0:
                        walk(i + 1, phi / math.sqrt(q), w * q, creg)
                elif p > 0:    # Pauli: branch weight is the listed prob.
                    walk(i + 1, phi, w * p, creg)
        elif k in _NON_GATES:
            qs = op["qubits"]
            m = len(qs)
            for pat in range(1 << m):
                P, R = full[i][pat]
                phi = P @ psi
                q = float(np.vdot(phi, phi).real)
                if q <= 0:
                    continue
                phi = phi / math.sqrt(q)
                if k != "measure":
                    phi = R @ phi
                if k == "reset":
                    walk(i + 1, phi, w * q, creg)
                    continue
                for rec in range(1 << m):
                    c = 1.0
                    for t in range(m):
                        c *= _confusion((pat >> t) & 1, (rec >> t) & 1, ro)
                    if c > 0:
                        walk(i + 1, phi, w * q * c,
                             _set_bits(creg, op["clbits"], rec))
        else:
            walk(i + 1, full[i] @ psi, w, creg)

    psi0 = np.zeros(1 << n, dtype=complex)
    psi0[0] = 1.0
    walk(0, psi0, 1.0, 0)
    return out


def tvd(p: Dict[int, float], q: Dict[int, float]) -> float:
    keys = set(p) | set(q)
    return 0.5 * sum(abs(p.get(k, 0.0) - q.get(k, 0.0)) for k in keys)
