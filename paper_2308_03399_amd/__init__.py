"""Python binding of libsvbatch (MI355X multi-shot noisy state-vector
simulation). Argument marshalling only: every step of a run executes in the
library's HIP kernels. PyTorch supplies the device arena and the stream.

The raw C-ABI calls are exposed under their C names (``sv_batch_create``,
``sv_run_circuit``, ``sv_sample_counts``, ...); they raise ``SvError`` on a
non-zero status. ``marshal`` turns a plain-Python circuit / noise-model
description (see ``workloads``) into the ABI's structs, and ``Simulator``
bundles create/attach/run for convenience.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsvbatch.so")

SV_C64, SV_C128 = 0, 1
SV_MODE_BATCH, SV_MODE_BRANCH, SV_MODE_PLAIN = 0, 1, 2
STATUS = {0: "SV_OK", 1: "SV_EINVAL", 2: "SV_ENOMEM", 3: "SV_EDEVICE",
          4: "SV_ESTATE", 5: "SV_EUNSUPPORTED"}
OP_KIND = {"id": 1, "x": 2, "y": 3, "z": 4, "h": 5, "s": 6, "sdg": 7, "t": 8,
           "tdg": 9, "u3": 10, "cx": 20, "cz": 21, "swap": 22, "unitary": 30,
           "measure": 40, "reset": 41, "measure_reset": 42, "bfunc": 45}
PAULI_CODE = {"I": 0, "X": 1, "Y": 2, "Z": 3}
MAX_INLINE = 8

EXPORTED = ["sv_batch_create", "sv_batch_footprint", "sv_batch_attach",
            "sv_batch_set_option", "sv_run_circuit", "sv_run_sweep",
            "sv_run_circuit_noalloc", "sv_sample_counts",
            "sv_get_memory", "sv_get_margins", "sv_get_state", "sv_get_stats",
            "sv_batch_destroy", "sv_last_error"]


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class sv_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("nq", ctypes.c_uint32),
                ("q", ctypes.c_uint32 * MAX_INLINE),
                ("c", ctypes.c_uint32 * MAX_INLINE),
                ("p", ctypes.c_double * 3),
                ("mat", ctypes.POINTER(ctypes.c_double)),
                ("q_ext", ctypes.POINTER(ctypes.c_uint32)),
                ("c_ext", ctypes.POINTER(ctypes.c_uint32)),
                ("cond_mask", ctypes.c_uint64), ("cond_value", ctypes.c_uint64)]


class sv_pauli_channel(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_uint32), ("n_terms", ctypes.c_uint32),
                ("prob", ctypes.POINTER(ctypes.c_double)),
                ("pauli", ctypes.POINTER(ctypes.c_uint8))]


class sv_kraus_channel(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_uint32), ("n_mats", ctypes.c_uint32),
                ("mats", ctypes.POINTER(ctypes.c_double))]


class sv_noise_rule(ctypes.Structure):
    _fields_ = [("gate_kinds_mask", ctypes.c_uint64),
                ("is_kraus", ctypes.c_uint32), ("channel", ctypes.c_void_p)]


class sv_noise_model(ctypes.Structure):
    _fields_ = [("n_rules", ctypes.c_uint32),
                ("rules", ctypes.POINTER(sv_noise_rule)),
                ("readout_p01", ctypes.c_double),
                ("readout_p10", ctypes.c_double)]


class sv_stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("passes", ctypes.c_uint64),
                ("amp_bytes", ctypes.c_uint64), ("reductions", ctypes.c_uint64),
                ("branches", ctypes.c_uint64), ("restarts", ctypes.c_uint64),
                ("waiting_shots", ctypes.c_uint64),
                ("expanded_ops", ctypes.c_uint64),
                ("gate_count", ctypes.c_uint64), ("workers", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("tile_qubits", ctypes.c_uint32),
                ("static_passes", ctypes.c_uint32), ("flops", ctypes.c_uint64),
                ("exec_ms", ctypes.c_double), ("exec_launches", ctypes.c_uint32),
                ("tile_buffers", ctypes.c_uint32), ("groups", ctypes.c_uint64),
                ("uops", ctypes.c_uint64), ("near_ties", ctypes.c_uint64),
                ("graph_replays", ctypes.c_uint32), ("program_uploads", ctypes.c_uint32),
                ("mfma", ctypes.c_uint32)]

    def as_dict(self) -> Dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library. Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_2308_03399_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    U64 = ctypes.c_uint64
    L.sv_batch_create.argtypes = [ctypes.c_int, I64, ctypes.c_int,
                                  ctypes.POINTER(P)]
    L.sv_batch_footprint.argtypes = [P, ctypes.POINTER(U64), ctypes.POINTER(U64)]
    L.sv_batch_attach.argtypes = [P, P, U64, P]
    L.sv_batch_set_option.argtypes = [P, ctypes.c_char_p, I64]
    L.sv_run_circuit.argtypes = [P, ctypes.POINTER(sv_op), ctypes.c_size_t,
                                 ctypes.POINTER(sv_noise_model), U64]
    L.sv_run_sweep.argtypes = [P, ctypes.POINTER(sv_op), ctypes.c_size_t,
                               ctypes.POINTER(sv_noise_model), U64, P, ctypes.c_size_t]
    L.sv_run_circuit_noalloc.argtypes = [P, ctypes.POINTER(sv_op), ctypes.c_size_t,
                                         ctypes.POINTER(sv_noise_model), U64, P, P,
                                         ctypes.c_size_t]
    L.sv_sample_counts.argtypes = [P, P, P, ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_size_t)]
    L.sv_get_memory.argtypes = [P, P, ctypes.c_size_t]
    L.sv_get_margins.argtypes = [P, P, ctypes.c_size_t]
    L.sv_get_state.argtypes = [P, P, ctypes.c_size_t]
    L.sv_get_stats.argtypes = [P, ctypes.POINTER(sv_stats)]
    L.sv_batch_destroy.argtypes = [P]
    for name in EXPORTED[:-1]:
        getattr(L, name).restype = ctypes.c_int
    L.sv_last_error.restype = ctypes.c_char_p
    L.sv_last_error.argtypes = []
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise SvError(status, lib().sv_last_error().decode(errors="replace"))


# ---------------------------------------------------------------- C names
def sv_batch_create(n_qubits: int, n_shots: int, dtype: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().sv_batch_create(int(n_qubits), int(n_shots), int(dtype),
                                 ctypes.byref(h)))
    return h.value


def sv_batch_set_option(h: int, key: str, value: int):
    _check(lib().sv_batch_set_option(h, key.encode(), int(value)))


def sv_batch_footprint(h: int):
    req = ctypes.c_uint64()
    per = ctypes.c_uint64()
    _check(lib().sv_batch_footprint(h, ctypes.byref(req), ctypes.byref(per)))
    return req.value, per.value


def sv_batch_attach(h: int, arena_ptr: int, arena_bytes: int, stream: int):
    _check(lib().sv_batch_attach(h, arena_ptr, arena_bytes, stream))


def sv_run_circuit(h: int, marshalled, seed: int):
    ops, n_ops, nm = marshalled["ops"], marshalled["n_ops"], marshalled["nm"]
    _check(lib().sv_run_circuit(h, ops, n_ops, nm, int(seed)))


def sv_run_sweep(h: int, marshalled, seed: int, params) -> None:
    """params: array (n_sets, n_u3, 3) of U3 angles, one row per set."""
    ops, n_ops, nm = marshalled["ops"], marshalled["n_ops"], marshalled["nm"]
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    if a.ndim != 3 or a.shape[2] != 3:
        raise ValueError("params must have shape (n_sets, n_u3, 3)")
    _check(lib().sv_run_sweep(h, ops, n_ops, nm, int(seed), a.ctypes.data, a.shape[0]))


def sv_run_circuit_noalloc(h: int, marshalled, seed: int, stream: int,
                           n_shots: int) -> np.ndarray:
    """The run of sv_run_circuit on the library's own device buffer (the
    handle is not attached); returns the per-shot registers."""
    ops, n_ops, nm = marshalled["ops"], marshalled["n_ops"], marshalled["nm"]
    out = np.zeros(n_shots, dtype=np.uint64)
    _check(lib().sv_run_circuit_noalloc(h, ops, n_ops, nm, int(seed), stream,
                                        out.ctypes.data, n_shots))
    return out


def sv_sample_counts(h: int, capacity: int = 0) -> Dict[int, int]:
    """(key -> count) of the last run. With capacity >= the number of
    distinct keys (the shot count always is) the histogram is computed once;
    with capacity 0 the size is queried first."""
    n = ctypes.c_size_t(0)
    cap = int(capacity)
    if cap <= 0:
        st = lib().sv_sample_counts(h, None, None, 0, ctypes.byref(n))
        if st not in (0, 1):
            _check(st)
        cap = max(int(n.value), 1)
    keys = np.zeros(cap, dtype=np.uint64)
    counts = np.zeros(cap, dtype=np.uint64)
    _check(lib().sv_sample_counts(h, keys.ctypes.data, counts.ctypes.data, cap,
                                  ctypes.byref(n)))
    return {int(k): int(c) for k, c in zip(keys[:n.value], counts[:n.value])}


def sv_get_memory(h: int, n_shots: int) -> np.ndarray:
    out = np.zeros(n_shots, dtype=np.uint64)
    _check(lib().sv_get_memory(h, out.ctypes.data, n_shots))
    return out


def sv_get_margins(h: int, n_shots: int) -> np.ndarray:
    out = np.zeros(n_shots, dtype=np.float64)
    _check(lib().sv_get_margins(h, out.ctypes.data, n_shots))
    return out


def sv_get_state(h: int, n_qubits: int) -> np.ndarray:
    out = np.zeros(2 << n_qubits, dtype=np.float64)
    _check(lib().sv_get_state(h, out.ctypes.data, 1 << n_qubits))
    return out.view(np.complex128)


def sv_get_stats(h: int) -> Dict:
    s = sv_stats()
    _check(lib().sv_get_stats(h, ctypes.byref(s)))
    return s.as_dict()


def sv_batch_destroy(h: int):
    _check(lib().sv_batch_destroy(h))


def sv_last_error() -> str:
    return lib().sv_last_error().decode(errors="replace")


# ---------------------------------------------------------------- marshalling
def marshal(circuit: Dict, noise: Optional[Dict]) -> Dict:
    """Build the ABI structs for a circuit / noise-model description. The
    returned dict keeps every buffer alive while it is referenced."""
    keep = []
    ops = circuit["ops"]
    arr = (sv_op * max(len(ops), 1))()
    for i, op in enumerate(ops):
        o = arr[i]
        o.kind = OP_KIND[op["kind"]]
        qs = [int(q) for q in op.get("qubits", [])]
        cs = [int(c) for c in op.get("clbits", [])]
        o.nq = len(qs)
        if len(qs) <= MAX_INLINE:
            for t, q in enumerate(qs):
                o.q[t] = q
            for t, c in enumerate(cs):
                o.c[t] = c
        else:
            qa = (ctypes.c_uint32 * len(qs))(*qs)
            ca = (ctypes.c_uint32 * max(len(cs), 1))(*(cs or [0]))
            keep += [qa, ca]
            o.q_ext = ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint32))
            o.c_ext = ctypes.cast(ca, ctypes.POINTER(ctypes.c_uint32))
        for t, p in enumerate(op.get("params", [])):
            o.p[t] = float(p)
        if op["kind"] == "bfunc":
            o.cond_mask, o.cond_value = int(op["mask"]), int(op["value"])
        elif op.get("cond"):
            o.cond_mask, o.cond_value = int(op["cond"][0]), int(op["cond"][1])
        if op["kind"] == "unitary":
            m = np.asarray(op["matrix"], dtype=np.complex128)
            flat = np.ascontiguousarray(np.stack([m.real, m.imag], -1).ravel())
            keep.append(flat)
            o.mat = flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nm_ptr = None
    if noise is not None:
        rules = noise.get("rules", [])
        rarr = (sv_noise_rule * max(len(rules), 1))()
        for r, ru in enumerate(rules):
            mask = 0
            for g in ru["gates"]:
                mask |= 1 << OP_KIND[g]
            rarr[r].gate_kinds_mask = mask
            if ru["type"] == "pauli":
                probs = np.asarray(ru["probs"], dtype=np.float64)
                codes = np.asarray([PAULI_CODE[ch] for s in ru["paulis"] for ch in s],
                                   dtype=np.uint8)
                ch = sv_pauli_channel(ru["nq"], len(probs),
                                      probs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
                keep += [probs, codes, ch]
                rarr[r].is_kraus = 0
            else:
                mats = np.asarray(ru["mats"], dtype=np.complex128)
                flat = np.ascontiguousarray(np.stack([mats.real, mats.imag], -1).ravel())
                ch = sv_kraus_channel(ru["nq"], len(mats),
                                      flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
                keep += [flat, ch]
                rarr[r].is_kraus = 1
            rarr[r].channel = ctypes.cast(ctypes.pointer(ch), ctypes.c_void_p)
        ro = noise.get("readout", [0.0, 0.0])
        nm = sv_noise_model(len(rules), ctypes.cast(rarr, ctypes.POINTER(sv_noise_rule)),
                            float(ro[0]), float(ro[1]))
        keep += [rarr, nm]
        nm_ptr = ctypes.pointer(nm)
    return {"ops": arr, "n_ops": len(ops), "nm": nm_ptr, "keep": keep}


# ---------------------------------------------------------------- convenience
class Simulator:
    """One handle with its torch-owned device arena on the current stream."""

    def __init__(self, n_qubits: int, n_shots: int, dtype: str = "c64",
                 mode: str = "batch", device: str = "cuda:0", **options):
        import torch
        self.torch = torch
        self.n_qubits = n_qubits
        self.n_shots = n_shots
        self.h = sv_batch_create(n_qubits, n_shots,
                                 SV_C128 if dtype == "c128" else SV_C64)
        sv_batch_set_option(self.h, "mode",
                            {"batch": SV_MODE_BATCH, "branch": SV_MODE_BRANCH,
                             "plain": SV_MODE_PLAIN}[mode])
        for k, v in options.items():
            sv_batch_set_option(self.h, k, int(v))
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            req, self.state_bytes = sv_batch_footprint(self.h)
            self.arena = torch.empty(int(req), dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            sv_batch_attach(self.h, self.arena.data_ptr(), int(req),
                            self.stream.cuda_stream)
        self.footprint = int(req)

    def run(self, circuit: Dict, noise: Optional[Dict], seed: int = 0):
        m = marshal(circuit, noise)
        with self.torch.cuda.device(self.device):
            sv_run_circuit(self.h, m, seed)

    def run_sweep(self, circuit: Dict, noise: Optional[Dict], params, seed: int = 0):
        m = marshal(circuit, noise)
        with self.torch.cuda.device(self.device):
            sv_run_sweep(self.h, m, seed, params)

    def counts(self, capacity: int = 0) -> Dict[int, int]:
        return sv_sample_counts(self.h, capacity or self.n_shots)

    def memory(self) -> np.ndarray:
        return sv_get_memory(self.h, self.n_shots)

    def margins(self) -> np.ndarray:
        return sv_get_margins(self.h, self.n_shots)

    def state(self) -> np.ndarray:
        return sv_get_state(self.h, self.n_qubits)

    def stats(self) -> Dict:
        return sv_get_stats(self.h)

    def close(self):
        if self.h:
            sv_batch_destroy(self.h)
            self.h = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
