"""Helpers for GPU tests: run a circuit through the C ABI and compare with
the FP64 oracle."""
import sys

import numpy as np

import oracle
from paper_2308_03399_amd import Simulator

SPIN_MS = 60000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(circ, noise, shots, dtype="c128", mode="batch", seed=0,
            dump_shot=None, want_margins=False, **opts):
    opts.setdefault("spin_limit_ms", SPIN_MS)
    if dump_shot is not None:
        opts["dump_shot"] = dump_shot
    sim = Simulator(circ["n_qubits"], shots, dtype=dtype, mode=mode, **opts)
    try:
        sim.run(circ, noise, seed=seed)
        mem = sim.memory()
        st = sim.stats()
        counts = sim.counts()
        state = sim.state() if dump_shot is not None else None
        margins = sim.margins() if want_margins else None
    finally:
        sim.close()
    return {"memory": mem, "stats": st, "counts": counts, "state": state, "margins": margins}


def oracle_memory(circ, noise, shots, seed=0):
    return oracle.run(circ, noise, shots, seed=seed)


def mismatches(a, b):
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    return int(np.sum(a != b))


def tvd_counts(mem_a, mem_b):
    ka, ca = np.unique(np.asarray(mem_a, dtype=np.uint64), return_counts=True)
    kb, cb = np.unique(np.asarray(mem_b, dtype=np.uint64), return_counts=True)
    pa = dict(zip(ka.tolist(), (ca / ca.sum()).tolist()))
    pb = dict(zip(kb.tolist(), (cb / cb.sum()).tolist()))
    keys = set(pa) | set(pb)
    return 0.5 * sum(abs(pa.get(k, 0) - pb.get(k, 0)) for k in keys)
