"""Run one sv_run_circuit of a named workload (for profilers): prints the
library's stats as one JSON line.

    python -m paper_2308_03399_amd.profile_run --workload c3_20q --shots 2048
"""
import argparse
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3_20q")
    ap.add_argument("--shots", type=int, default=2048)
    ap.add_argument("--dtype", default=None)
    ap.add_argument("--mode", default="batch", choices=["batch", "branch"])
    ap.add_argument("--tile-qubits", type=int, default=0)
    args = ap.parse_args()
    import workloads as W
    from paper_2308_03399_amd import Simulator
    w = W.workload(args.workload)
    dtype = args.dtype or w["dtype"]
    opts = {"tile_qubits": args.tile_qubits} if args.tile_qubits else {}
    sim = Simulator(w["circuit"]["n_qubits"], args.shots, dtype=dtype, mode=args.mode, **opts)
    sim.run(w["circuit"], w["noise"], seed=w["seed"])
    sim.counts()
    st = sim.stats()
    st.update({"workload": args.workload, "shots": args.shots, "dtype": dtype, "mode": args.mode})
    print(json.dumps(st), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
