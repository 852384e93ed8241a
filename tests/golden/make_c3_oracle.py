#!/usr/bin/env python3
"""Writes c3_oracle_registers.txt: the FP64 oracle's per-shot classical
registers and smallest decision margins for 256 shot ids of the 20-qubit,
60-layer noisy workload (random U3 + CX layers, depolarizing 1e-3 / 1e-2,
amplitude damping 5e-3, readout 2%; Philox seed 0), spread over the whole
100,000-shot job: 16 blocks of 16 consecutive ids starting at multiples of
6,250, the last block ending at id 99,999.

Calls only the oracle (oracle/traj.c) and the seeded input generators
(workloads/); about 20 core-minutes.

    python tests/golden/make_c3_oracle.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_registers.txt")
BLOCK = 16


def shot_ids():
    starts = [b * 6250 for b in range(15)] + [100_000 - BLOCK]
    return [s + i for s in starts for i in range(BLOCK)]


def main():
    w = W.workload("c3_20q")
    ids = shot_ids()
    t0 = time.time()
    mem, marg = oracle.run(w["circuit"], w["noise"], ids, seed=w["seed"], want_margins=True)
    dt = time.time() - t0
    with open(OUT, "w") as f:
        f.write("# FP64 oracle (oracle/traj.c) on the 20-qubit x 60-layer noisy workload,\n")
        f.write("# Philox seed %d, written by tests/golden/make_c3_oracle.py\n" % w["seed"])
        f.write("# columns: shot id, classical register (hex), smallest relative decision margin\n")
        for s, m, g in zip(ids, mem, marg):
            f.write("%d %x %.17g\n" % (s, int(m), float(g)))
    print(f"{len(ids)} shots in {dt:.0f} s -> {OUT}")


if __name__ == "__main__":
    main()
