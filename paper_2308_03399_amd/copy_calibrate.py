"""A plain device copy of a known size (torch's copy kernel), used to scale
the FETCH_SIZE / WRITE_SIZE hardware counters to bytes:

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2308_03399_amd.copy_calibrate --mib 1024
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.mib} MiB x {args.reps}", flush=True)


if __name__ == "__main__":
    main()
