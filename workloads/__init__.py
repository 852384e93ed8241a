"""Seeded synthetic inputs: circuits, noise models and request streams.

This module only *describes* inputs. It holds none of the simulation
arithmetic: no gate matrices, no noise-site expansion, no random draws of the
trajectory method. Both the product library (through its Python binding) and
the FP64 oracle consume the plain-Python descriptions built here.

Circuit description (plain data)::

    {"n_qubits": n, "n_clbits": c,
     "ops": [{"kind": "u3", "qubits": [q], "params": [theta, phi, lam]},
             {"kind": "cx", "qubits": [control, target]},
             {"kind": "unitary", "qubits": [q0, q1], "matrix": [[...]]},
             {"kind": "measure", "qubits": [...], "clbits": [...]},
             {"kind": "measure_reset", "qubits": [...], "clbits": [...]},
             {"kind": "reset", "qubits": [...]}, ...]}

Noise model description::

    {"rules": [{"gates": ["u3"], "type": "pauli", "nq": 1,
                "probs": [...], "paulis": ["I", "X", "Y", "Z"]},
               {"gates": ["u3"], "type": "kraus", "nq": 1,
                "mats": [[[a, b], [c, d]], ...]}],
     "readout": [p01, p10]}

A rule is attached after every gate whose kind is listed and whose qubit
count equals the rule's ``nq``, on that gate's qubits, in rule order
(the all-qubit error rules of the paper's noise-model example, Sec. III-B).
In a Pauli string, character ``t`` acts on the gate's qubit ``t``.

The synthetic workloads follow the paper's setting (random noisy circuits,
many shots, Sec. V) with seeded random layered circuits standing in for the
paper's QFT runs, whose figures are not available.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

GATE_KINDS_1Q = ("id", "x", "y", "z", "h", "s", "sdg", "t", "tdg", "u3")
GATE_KINDS_2Q = ("cx", "cz", "swap")
NONUNITARY_KINDS = ("measure", "reset", "measure_reset")

PAULI_CHARS = "IXYZ"


# ----------------------------------------------------------------------------
# Noise channels (inputs: the user's noise model)
# ----------------------------------------------------------------------------

def depolarizing_pauli(p: float, nq: int) -> Dict:
    """Pauli-channel form of the n-qubit depolarizing channel
    E(rho) = (1-p) rho + p I/2^n, listed as (probability, Pauli string).

    Every one of the 4^n Pauli strings carries p/4^n, the identity gets
    1 - p + p/4^n. Strings are ordered by their base-4 code with the gate's
    qubit 0 as the least-significant digit, I=0 X=1 Y=2 Z=3.
    """
    n_terms = 4 ** nq
    probs = []
    paulis = []
    for code in range(n_terms):
        chars = []
        c = code
        for _ in range(nq):
            chars.append(PAULI_CHARS[c % 4])
            c //= 4
        paulis.append("".join(chars))
        probs.append(p / n_terms + (1.0 - p if code == 0 else 0.0))
    return {"type": "pauli", "nq": nq, "probs": probs, "paulis": paulis}


def haar_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary (QR of a complex Gaussian matrix, phases fixed)."""
    z = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_kraus(nq: int, n_mats: int, seed: int) -> Dict:
    """Random n-qubit Kraus channel of n_mats matrices: the blocks of a
    random isometry (QR of a (n_mats*2^nq) x 2^nq complex Gaussian), so
    sum_j K_j^dagger K_j = I."""
    rng = np.random.default_rng(seed)
    d = 1 << nq
    z = rng.normal(size=(n_mats * d, d)) + 1j * rng.normal(size=(n_mats * d, d))
    v, _ = np.linalg.qr(z)
    return {"type": "kraus", "nq": nq,
            "mats": [v[j * d:(j + 1) * d, :].tolist() for j in range(n_mats)]}


def random_pauli_channel(nq: int, seed: int, p_noise: float = 0.3) -> Dict:
    """Random n-qubit Pauli channel over all 4^nq strings (base-4 order as
    in depolarizing_pauli): identity 1 - p_noise, the rest split by random
    weights."""
    rng = np.random.default_rng(seed)
    base = depolarizing_pauli(0.0, nq)
    w = rng.random(4 ** nq - 1)
    probs = [1.0 - p_noise] + list(p_noise * w / w.sum())
    return {"type": "pauli", "nq": nq, "probs": probs, "paulis": base["paulis"]}


def random_dense(n_qubits: int, n_ops: int, seed: int, widths=(3, 4, 5),
                 n_mid: int = 0) -> Dict:
    """Random circuit of dense unitaries on `widths` qubits mixed with U3
    and CX gates, optional mid-circuit measures, final measure of all
    qubits."""
    rng = np.random.default_rng(seed)
    ops: List[Dict] = []
    n_cl = n_qubits
    mid_at = set(rng.choice(n_ops, size=min(n_mid, n_ops), replace=False).tolist()) if n_mid else set()
    for i in range(n_ops):
        k = int(rng.integers(3))
        if k == 0:
            w = int(rng.choice([x for x in widths if x <= n_qubits]))
            qs = [int(x) for x in rng.choice(n_qubits, w, replace=False)]
            ops.append({"kind": "unitary", "qubits": qs,
                        "matrix": haar_unitary(1 << w, rng).tolist()})
        elif k == 1:
            ops.append({"kind": "u3", "qubits": [int(rng.integers(n_qubits))],
                        "params": [float(x) for x in rng.uniform(0, 2 * math.pi, 3)]})
        else:
            a, b = (int(x) for x in rng.choice(n_qubits, 2, replace=False))
            ops.append({"kind": "cx", "qubits": [a, b]})
        if i in mid_at:
            q = int(rng.integers(n_qubits))
            ops.append({"kind": "measure", "qubits": [q], "clbits": [n_cl]})
            n_cl += 1
    ops.append({"kind": "measure", "qubits": list(range(n_qubits)),
                "clbits": list(range(n_qubits))})
    return {"n_qubits": n_qubits, "n_clbits": n_cl, "ops": ops}


def pauli_table(probs: Sequence[float], paulis: Sequence[str]) -> Dict:
    nq = len(paulis[0])
    return {"type": "pauli", "nq": nq, "probs": list(map(float, probs)),
            "paulis": list(paulis)}


def amplitude_damping_kraus(gamma: float) -> Dict:
    """Kraus form of single-qubit amplitude damping with decay gamma."""
    k0 = [[1.0, 0.0], [0.0, math.sqrt(1.0 - gamma)]]
    k1 = [[0.0, math.sqrt(gamma)], [0.0, 0.0]]
    return {"type": "kraus", "nq": 1, "mats": [k0, k1]}


def depolarizing_kraus(p: float, nq: int) -> Dict:
    """Kraus form of the same n-qubit depolarizing channel as
    depolarizing_pauli: sqrt(prob) times each Pauli string, in the same
    order (any channel, Pauli ones included, can be given as a Kraus list,
    Sec. III-B). Matrix index bit t is the gate's qubit t."""
    single = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]),
              "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.diag([1, -1])}
    pc = depolarizing_pauli(p, nq)
    mats = []
    for prob, s in zip(pc["probs"], pc["paulis"]):
        m = np.ones((1, 1), dtype=complex)
        for ch in s:                      # qubit 0 first: it ends up least significant
            m = np.kron(single[ch], m)
        mats.append((math.sqrt(prob) * m).tolist())
    return {"type": "kraus", "nq": nq, "mats": mats}


def qft(n_qubits: int, prepare: int = 0, measure_all: bool = True) -> Dict:
    """Textbook quantum Fourier transform (Sec. V workload) written over the
    gate set the paper's noise model names: H, phase (U3(0, 0, lam)) and CX.
    Each controlled phase CP(lam) on (a, b) is p(lam/2) a, CX(a, b),
    p(-lam/2) b, CX(a, b), p(lam/2) b; the final qubit reversal is three CX
    per swap. `prepare` sets the input basis state with X gates first."""
    ops = []
    for q in range(n_qubits):
        if (prepare >> q) & 1:
            ops.append({"kind": "x", "qubits": [q]})

    def phase(q, lam):
        ops.append({"kind": "u3", "qubits": [q], "params": [0.0, 0.0, lam]})

    for j in reversed(range(n_qubits)):
        ops.append({"kind": "h", "qubits": [j]})
        for k in reversed(range(j)):
            lam = math.pi / (1 << (j - k))
            phase(k, lam / 2)
            ops.append({"kind": "cx", "qubits": [k, j]})
            phase(j, -lam / 2)
            ops.append({"kind": "cx", "qubits": [k, j]})
            phase(j, lam / 2)
    for i in range(n_qubits // 2):
        a, b = i, n_qubits - 1 - i
        ops += [{"kind": "cx", "qubits": [a, b]}, {"kind": "cx", "qubits": [b, a]},
                {"kind": "cx", "qubits": [a, b]}]
    if measure_all:
        ops.append({"kind": "measure", "qubits": list(range(n_qubits)),
                    "clbits": list(range(n_qubits))})
    return {"n_qubits": n_qubits, "ops": ops}


def qft_noise(p: float = 0.01, form: str = "pauli") -> Dict:
    """1% depolarizing noise after every one-qubit (H, phase) and two-qubit
    (CX) gate, as a Pauli channel or as the equivalent Kraus list."""
    make = depolarizing_pauli if form == "pauli" else depolarizing_kraus
    return noise_model([rule(["u3", "h", "x"], make(p, 1)), rule(["cx"], make(p, 2))])


def kraus_channel(mats: Sequence) -> Dict:
    mats = [np.asarray(m, dtype=complex).tolist() for m in mats]
    nq = int(round(math.log2(len(mats[0]))))
    return {"type": "kraus", "nq": nq, "mats": mats}


def noise_model(rules: Sequence[Dict] = (), readout=(0.0, 0.0)) -> Dict:
    return {"rules": [dict(r) for r in rules],
            "readout": [float(readout[0]), float(readout[1])]}


def rule(gates: Sequence[str], channel: Dict) -> Dict:
    r = dict(channel)
    r["gates"] = list(gates)
    return r


# ----------------------------------------------------------------------------
# Random layered circuits
# ----------------------------------------------------------------------------

def random_layered(n_qubits: int, n_layers: int, seed: int = 0,
                   two_qubit: str = "cx", measure_all: bool = True,
                   mid_measure=None) -> Dict:
    """Seeded random layered circuit.

    Per layer: U3 on qubits 0..n-1 in order with angles drawn uniformly in
    [0, 2pi), then a random permutation pi of the qubits and the two-qubit
    gate on (pi[2k], pi[2k+1]) for k < n//2 (first entry is the control).

    ``mid_measure``: optional (every, qubits) -- after every ``every``-th
    layer, a measure-and-reset of ``qubits``, recorded into clbits placed
    after the n final-measure clbits.
    """
    rng = np.random.default_rng(seed)
    ops: List[Dict] = []
    n_clbits = n_qubits if measure_all else 0
    mid_every, mid_qubits = (mid_measure if mid_measure else (0, ()))
    next_mid_clbit = n_qubits
    for layer in range(n_layers):
        angles = rng.uniform(0.0, 2.0 * math.pi, size=(n_qubits, 3))
        for q in range(n_qubits):
            ops.append({"kind": "u3", "qubits": [q],
                        "params": [float(a) for a in angles[q]]})
        perm = rng.permutation(n_qubits)
        for k in range(n_qubits // 2):
            ops.append({"kind": two_qubit,
                        "qubits": [int(perm[2 * k]), int(perm[2 * k + 1])]})
        if mid_every and (layer + 1) % mid_every == 0:
            cl = list(range(next_mid_clbit, next_mid_clbit + len(mid_qubits)))
            next_mid_clbit += len(mid_qubits)
            ops.append({"kind": "measure_reset", "qubits": list(mid_qubits),
                        "clbits": cl})
    n_clbits = max(n_clbits, next_mid_clbit) if mid_every else n_clbits
    if measure_all:
        ops.append({"kind": "measure", "qubits": list(range(n_qubits)),
                    "clbits": list(range(n_qubits))})
    return {"n_qubits": n_qubits, "n_clbits": n_clbits, "ops": ops}


def count_gates(circuit: Dict) -> int:
    """Original gates counted by the throughput metric (U3 and 2q gates;
    noise, measure and reset excluded)."""
    return sum(1 for op in circuit["ops"]
               if op["kind"] in GATE_KINDS_1Q + GATE_KINDS_2Q + ("unitary",))


# ----------------------------------------------------------------------------
# The five benchmark workloads
# ----------------------------------------------------------------------------

def depol_model(p1: float = 1e-3, p2: float = 1e-2, gates1=("u3",),
                gates2=("cx",), extra_rules=(), readout=(0.0, 0.0)) -> Dict:
    rules = [rule(gates1, depolarizing_pauli(p1, 1))]
    rules += list(extra_rules)
    rules.append(rule(gates2, depolarizing_pauli(p2, 2)))
    return noise_model(rules, readout)


def workload(name: str) -> Dict:
    """Returns {"circuit", "noise", "shots", "dtype", "seed", ...} for one of
    the named workloads."""
    if name == "c1_10q":
        return {"name": name,
                "circuit": random_layered(10, 20, seed=0),
                "noise": depol_model(),
                "shots": 1000, "dtype": "c128", "seed": 0}
    if name == "c2_16q":
        return {"name": name,
                "circuit": random_layered(16, 40, seed=0,
                                          mid_measure=(10, (0, 1))),
                "noise": depol_model(),
                "shots": 10_000, "dtype": "c128", "seed": 0}
    if name == "c3_20q":
        ad = rule(("u3",), amplitude_damping_kraus(5e-3))
        # depolarizing then amplitude damping after each U3, depolarizing
        # after each CX (rule order gives the insertion order)
        rules = [rule(("u3",), depolarizing_pauli(1e-3, 1)), ad,
                 rule(("cx",), depolarizing_pauli(1e-2, 2))]
        return {"name": name,
                "circuit": random_layered(20, 60, seed=0),
                "noise": noise_model(rules, readout=(0.02, 0.02)),
                "shots": 100_000, "dtype": "c64", "seed": 0}
    if name == "c4_26q":
        return {"name": name,
                "circuit": random_layered(26, 80, seed=0, two_qubit="cz"),
                "noise": depol_model(gates2=("cz",)),
                "shots": 2000, "dtype": "c64", "seed": 0}
    raise KeyError(name)


def serving_stream(n_requests: int, rate_per_s: float, seed: int = 0,
                   qubit_range=(8, 24), depth_range=(10, 60),
                   shots_range=(100, 100_000)) -> List[Dict]:
    """Poisson arrivals of random noisy U3+CX circuits. Request i uses
    circuit seed i; qubits and depth uniform, shots log-uniform."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(rng.integers(qubit_range[0], qubit_range[1] + 1))
        d = int(rng.integers(depth_range[0], depth_range[1] + 1))
        lo, hi = math.log(shots_range[0]), math.log(shots_range[1])
        shots = int(round(math.exp(rng.uniform(lo, hi))))
        out.append({"id": i, "arrival_s": t,
                    "circuit": random_layered(n, d, seed=i),
                    "noise": depol_model(), "shots": shots, "dtype": "c64",
                    "seed": i})
    return out


# ----------------------------------------------------------------------------
# Small circuits used by tests
# ----------------------------------------------------------------------------

def random_small(n_qubits: int, n_ops: int, seed: int, kinds=None,
                 measure_all: bool = True, n_mid: int = 0, p_cond: float = 0.0) -> Dict:
    """Random mixed circuit over the supported op kinds, for parity tests.
    With p_cond > 0, gates after a mid-circuit measure are made conditional
    on already written clbits with that probability, and each mid-circuit
    measure is followed by a branch op (bfunc) on a fresh clbit."""
    rng = np.random.default_rng(seed)
    crng = np.random.default_rng(seed + 7919)
    written: List[int] = []

    def maybe_cond(op):
        if p_cond > 0 and written and crng.random() < p_cond:
            bits = [int(b) for b in crng.choice(written, min(len(written), int(crng.integers(1, 3))),
                                                 replace=False)]
            mask = sum(1 << b for b in bits)
            value = sum((int(crng.integers(2)) << b) for b in bits)
            op["cond"] = [mask, value]
        return op
    kinds = kinds or ["u3", "h", "x", "y", "z", "s", "t", "sdg", "tdg",
                      "cx", "cz", "swap", "unitary2"]
    if n_qubits < 2:
        kinds = [k for k in kinds if k not in ("cx", "cz", "swap", "unitary2")]
    ops = []
    n_cl = n_qubits if measure_all else 0
    mid_at = set(rng.choice(n_ops, size=min(n_mid, n_ops), replace=False).tolist()) if n_mid else set()
    for i in range(n_ops):
        k = kinds[int(rng.integers(len(kinds)))]
        if k in GATE_KINDS_1Q:
            q = int(rng.integers(n_qubits))
            op = {"kind": k, "qubits": [q]}
            if k == "u3":
                op["params"] = [float(x) for x in rng.uniform(0, 2 * math.pi, 3)]
            ops.append(maybe_cond(op))
        elif k == "unitary2":
            a, b = (int(x) for x in rng.choice(n_qubits, 2, replace=False))
            z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
            qm, rm = np.linalg.qr(z)
            qm = qm * (np.diag(rm) / np.abs(np.diag(rm)))
            ops.append(maybe_cond({"kind": "unitary", "qubits": [a, b],
                                   "matrix": [[complex(v) for v in row] for row in qm]}))
        else:
            a, b = (int(x) for x in rng.choice(n_qubits, 2, replace=False))
            ops.append(maybe_cond({"kind": k, "qubits": [a, b]}))
        if i in mid_at:
            m = int(rng.integers(1, min(3, n_qubits) + 1))
            qs = [int(x) for x in rng.choice(n_qubits, m, replace=False)]
            cl = list(range(n_cl, n_cl + m))
            n_cl += m
            kind = "measure_reset" if rng.integers(2) else "measure"
            ops.append(maybe_cond({"kind": kind, "qubits": qs, "clbits": cl}))
            if p_cond > 0:
                written += cl
                bits = [int(b) for b in crng.choice(written, min(len(written), 2), replace=False)]
                ops.append({"kind": "bfunc", "clbits": [n_cl],
                            "mask": sum(1 << b for b in bits),
                            "value": sum((int(crng.integers(2)) << b) for b in bits)})
                written.append(n_cl)
                n_cl += 1
    if measure_all:
        ops.append({"kind": "measure", "qubits": list(range(n_qubits)),
                    "clbits": list(range(n_qubits))})
    return {"n_qubits": n_qubits, "n_clbits": n_cl, "ops": ops}
