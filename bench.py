#!/usr/bin/env python3
"""Throughput benchmark of the multi-shot noisy state-vector hot path.

Workload: 20 qubits, 60 layers of random U3 on every qubit + CX on a random
disjoint pairing; depolarizing noise p=1e-3 after U3 and 1e-2 after CX,
amplitude damping gamma=5e-3 after U3, 2% symmetric readout error; 100,000
shots; complex64 storage with FP64 decisions. A step is one wave of
shots_per_step consecutive shot ids (the default 10 steps x 10,000 shots is
the whole 100k-shot job), each wave being sv_run_circuit + sv_sample_counts
through the C ABI. Inputs are seeded and synthetic.

Prints one JSON line (rank 0, N=1). Only one GPU is supported.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "c1_10q": {"steps": 1, "warmup": 1, "shots_per_step": 1000, "plain_shots": 16, "dtype": "c128",
               "metric": "shots×gates/s, 10q noisy 1000 shots (states resident in LDS)",
               "describe": "c1_10q: 10 qubits x 20 layers random U3 + CX pairing; depolarizing "
                           "1e-3 (1q) / 1e-2 (2q); 1000 shots in one launch"},
    "c2_16q": {"steps": 1, "warmup": 1, "shots_per_step": 10_000, "plain_shots": 16,
               "dtype": "c128",
               "metric": "shots×gates/s and achieved HBM GB/s, 16q noisy 10k shots with "
                         "mid-circuit measure and reset",
               "describe": "c2_16q: 16 qubits x 40 layers random U3 + CX pairing; depolarizing "
                           "1e-3 (1q) / 1e-2 (2q); measure and reset of qubits 0, 1 every 10 "
                           "layers; 10,000 shots in one launch"},
    "c3_20q": {"steps": 10, "warmup": 1, "shots_per_step": 10_000, "plain_shots": 16,
               "dtype": "c64",
               "metric": "shots×gates/s and achieved HBM GB/s, 20q noisy 100k shots; c64 vs c128",
               "describe": "c3_20q: 20 qubits x 60 layers random U3 + CX pairing; depolarizing "
                           "1e-3 (1q) / 1e-2 (2q), amplitude damping 5e-3, readout 2%; "
                           "100,000 shots as waves"},
    "c4_26q": {"steps": 1, "warmup": 0, "shots_per_step": 2000, "plain_shots": 1,
               "dtype": "c64",
               "metric": "shots×gates/s and achieved HBM GB/s, 26q noisy 2000 shots",
               "describe": "c4_26q: 26 qubits x 80 layers random U3 + CZ pairing; depolarizing "
                           "1e-3 (1q) / 1e-2 (2q); 2000 shots in one launch"},
}
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TF = 157.3    # MI355X published FP32 vector
FP64_VECTOR_PEAK_TF = 78.6


def progress(msg: str):
    """One progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the executor's source and of the build script (its flags)."""
    h = hashlib.sha256()
    for f in ("csrc/kernels.hip", "csrc/kernels_mfma.hip", "csrc/program.h", "build.py"):
        with open(os.path.join(ROOT, "paper_2308_03399_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, dtype: str, shots_per_step: int, mode: str,
                     alg_bytes: int):
    """HBM bytes per executor launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source, in the same mode,
    with the same shots per launch and the same pass plan (its algorithmic
    bytes per launch equal this launch's)."""
    path = os.path.join(ROOT, "profiles", f"exec_kernel_{workload}_{dtype}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if int(t.get("shots_per_launch", -1)) != shots_per_step or t.get("mode", "batch") != mode:
        return None
    if int(t.get("algorithmic_bytes_per_launch", -1)) != int(alg_bytes):
        return None
    return float(t["hbm_bytes_per_launch"])


def cpu_baseline(circ, noise, gate_count: int, seed: int, job_shots: int, wave: int):
    """The FP64 oracle timed on the host cores: one shot per core, ids
    spread over the first wave (0..wave-1). Returns the baseline record and
    the oracle's registers and decision margins for those ids."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    shots = [k * (wave // cores) for k in range(cores)]
    t0 = time.perf_counter()
    mem, marg = oracle.run(circ, noise, shots, seed=seed, n_threads=cores, want_margins=True)
    dt = time.perf_counter() - t0
    rec = {"value": len(shots) * gate_count / dt, "unit": "shots*gates/s",
           "cores": cores, "kind": "oracle",
           "sample": f"{len(shots)} shot ids spread over 0..{wave - 1} of the same workload "
                     f"(one shot per core, {dt:.1f} s wall)",
           "full_job_estimate_s": round(job_shots * dt / len(shots), 1)}
    return rec, shots, mem, marg


def other_form(circ, noise, seed, gates, shots, dtype, mode, keep_memory=False, stats=False):
    """One timed wave of the same workload in another precision or form
    (shot ids 0..shots-1), for the comparisons the metric names."""
    import torch
    from paper_2308_03399_amd import Simulator
    sim = Simulator(circ["n_qubits"], shots, dtype=dtype, mode=mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(circ, noise, seed=seed)
    counts = sim.counts(capacity=shots)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = sim.stats()
    mem = sim.memory() if keep_memory else None
    sim.close()
    torch.cuda.empty_cache()
    assert sum(counts.values()) == shots
    out = {"dtype": dtype, "mode": mode, "shots": shots,
           "value": shots * gates / dt, "unit": "shots*gates/s",
           "ms": round(dt * 1e3, 1),
           "hbm_gbs": round(st["amp_bytes"] / (st["exec_ms"] * 1e-3) / 1e9, 1)
           if st["exec_ms"] > 0 else None,
           "passes_per_shot": round(st["passes"] / shots, 2)}
    if mode == "branch":
        out.update(slots=st["slots"], branches=st["branches"], restarts=st["restarts"])
    out["near_ties"] = st["near_ties"]
    if stats:
        out["stats"] = st
    return (out, mem) if keep_memory else out


def shot_state(circ, noise, seed, dtype, shot):
    """Normalised final state of one shot (complex128 copy)."""
    from paper_2308_03399_amd import Simulator
    sim = Simulator(circ["n_qubits"], 1, dtype=dtype, shot_offset=shot, dump_shot=0)
    try:
        sim.run(circ, noise, seed=seed)
        return sim.state()
    finally:
        sim.close()


def wave_memory(circ, noise, seed, shots, dtype):
    """Per-shot registers of shot ids 0..shots-1 (batch mode)."""
    from paper_2308_03399_amd import Simulator
    sim = Simulator(circ["n_qubits"], shots, dtype=dtype)
    try:
        sim.run(circ, noise, seed=seed)
        return sim.memory()
    finally:
        sim.close()


def c64_vs_fp64(mem64, mem128, circ, noise, seed, n_state_shots=64):
    """Complex64 path against the FP64 path on the same shot ids.

    * With the workload's readout error: per-shot agreement and the
      total-variation distance of the two count histograms (shared draws,
      so it is at most the disagreement rate).
    * With readout error off (the register is then the sampled basis
      index): each disagreement is split into a final sample that landed on
      the neighbouring index (u*N between the complex64 and FP64 running
      sums of one of the 2^n boundaries) and any other (a trajectory that
      went another way at a Kraus choice).
    * For n_state_shots shots spread over the wave: the TVD of the two
      output distributions the final measurement samples from, the largest
      amplitude error and the infidelity of the final states."""
    import numpy as np
    agree = float(np.mean(mem64 == mem128))
    k64, c64 = np.unique(mem64, return_counts=True)
    k128, c128 = np.unique(mem128, return_counts=True)
    p = dict(zip(k64.tolist(), (c64 / c64.sum()).tolist()))
    q = dict(zip(k128.tolist(), (c128 / c128.sum()).tolist()))
    tvd = 0.5 * sum(abs(p.get(k, 0.0) - q.get(k, 0.0)) for k in set(p) | set(q))
    B = int(mem64.size)
    noise0 = dict(noise, readout=[0.0, 0.0])
    a = wave_memory(circ, noise0, seed, B, "c64")
    b = wave_memory(circ, noise0, seed, B, "c128")
    diff = np.nonzero(a != b)[0]
    gap = np.abs(a[diff].astype(np.int64) - b[diff].astype(np.int64))
    adjacent = int(np.sum(gap == 1))
    tvds, errs, infid = [], [], []
    for k in range(n_state_shots):
        shot = k * (B // n_state_shots)
        if k % 8 == 0:
            progress(f"final states of shot {shot} ({k + 1}/{n_state_shots}), complex64 and FP64")
        sa = shot_state(circ, noise, seed, "c64", shot)
        sb = shot_state(circ, noise, seed, "c128", shot)
        pa, pb = np.abs(sa) ** 2, np.abs(sb) ** 2
        tvds.append(0.5 * float(np.sum(np.abs(pa / pa.sum() - pb / pb.sum()))))
        errs.append(float(np.max(np.abs(sa - sb))))
        fid = abs(np.vdot(sa, sb)) ** 2 / (np.vdot(sa, sa).real * np.vdot(sb, sb).real)
        infid.append(float(1.0 - fid))
    return {"shots": B, "agreement": agree, "tvd": tvd,
            "readout_off": {"disagreements": int(diff.size),
                            "adjacent_index": adjacent,
                            "other": int(diff.size) - adjacent,
                            "other_rate": (int(diff.size) - adjacent) / B},
            "final_states": {"shots": n_state_shots,
                             "output_tvd_mean": float(np.mean(tvds)),
                             "output_tvd_max": float(np.max(tvds)),
                             "max_amp_err": float(np.max(errs)),
                             "infidelity_max": float(np.max(infid))},
            "reference": "complex128 GPU path on the same shot ids (per-shot equal to "
                         "the FP64 oracle on sampled shots)"}


def one_launch(args):
    """One sv_run_circuit (+ counts) of a workload for a profiler: prints
    the library's stats as one JSON line."""
    import workloads as W
    from paper_2308_03399_amd import Simulator
    w = W.workload(args.workload)
    dtype = args.dtype or w["dtype"]
    opts = {"tile_qubits": args.tile_qubits} if args.tile_qubits else {}
    sim = Simulator(w["circuit"]["n_qubits"], args.one_launch, dtype=dtype, mode=args.mode, **opts)
    sim.run(w["circuit"], w["noise"], seed=w["seed"])
    sim.counts()
    st = sim.stats()
    st.update({"workload": args.workload, "shots": args.one_launch, "dtype": dtype,
               "mode": args.mode})
    sim.close()
    print(json.dumps(st), flush=True)


def copy_calibrate(mib: int, reps: int = 3):
    """A plain device copy of a known size (torch's copy kernel), whose
    FETCH_SIZE / WRITE_SIZE counter readings scale those counters to bytes."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


def error_ratio_sweep(qubits, probs, shots=4000, plain_shots=16):
    """The paper's error-ratio experiment (Sec. V-D): QFT with depolarizing
    noise of rate p after every gate, as a Pauli channel or as the
    equivalent Kraus list, 4000 shots; batched (batch mode) and branched
    forms in complex64 against the plain per-shot FP64 form (timed on its
    first shot ids; linear in shots). One JSON line per point."""
    import workloads as W
    for n in qubits:
        circ = W.qft(n)
        gates = W.count_gates(circ)
        for form in ("pauli", "kraus"):
            for p in probs:
                noise = W.qft_noise(p, form)
                other_form(circ, noise, 0, gates, min(shots, 256), "c64", "batch")  # warm-up
                ba = other_form(circ, noise, 0, gates, shots, "c64", "batch", stats=True)
                br = other_form(circ, noise, 0, gates, shots, "c64", "branch", stats=True)
                pl = other_form(circ, noise, 0, gates, plain_shots, "c128", "plain")
                plain_ms = pl["ms"] / plain_shots * shots
                line = {"experiment": "error_ratio", "workload": f"qft_{n}q", "noise": form,
                        "p": p, "shots": shots, "gates_per_shot": gates,
                        "batch_c64_ms": ba["ms"], "batch_passes_per_shot": ba["passes_per_shot"],
                        "batch_reductions_per_shot": round(ba["stats"]["reductions"] / shots, 3),
                        "branch_c64_ms": br["ms"], "branch_states": br["branches"] + 1,
                        "branch_passes_per_shot": br["passes_per_shot"],
                        "plain_fp64_ms": round(plain_ms, 1),
                        "batch_speedup_over_plain": round(plain_ms / ba["ms"], 1),
                        "branch_speedup_over_plain": round(plain_ms / br["ms"], 1)}
                print(json.dumps(line), flush=True)


def copy_ceiling_gbs(gib: int = 2, reps: int = 5) -> float:
    """Device-to-device copy bandwidth (read + write bytes / time): the
    attainable HBM rate beside the 8 TB/s peak."""
    import torch
    a = torch.empty(gib << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (gib << 30) * reps / (ms * 1e-3) / 1e9


def qft_comparison(n, shots=4000, p=0.01, plain_shots=40):
    """The paper's single-GPU experiment (Sec. V-B): QFT with 1% Pauli or
    Kraus noise, 4000 shots, the batched and branched forms against the
    plain per-shot form (timed on its first shot ids; linear in shots)."""
    import workloads as W
    circ = W.qft(n)
    gates = W.count_gates(circ)
    for form in ("pauli", "kraus"):
        noise = W.qft_noise(p, form)
        res = {}
        for dtype, mode in (("c64", "batch"), ("c128", "batch"), ("c64", "branch"),
                            ("c128", "branch")):
            other_form(circ, noise, 0, gates, min(shots, 256), dtype, mode)  # warm-up
            res[f"{dtype}_{mode}"] = other_form(circ, noise, 0, gates, shots, dtype, mode)
        pl = other_form(circ, noise, 0, gates, plain_shots, "c128", "plain")
        per_shot_ms = pl["ms"] / plain_shots
        line = {"workload": f"qft_{n}q", "noise": f"{form} 1%", "shots": shots,
                "gates_per_shot": gates,
                "plain_fp64_ms_for_all_shots": round(per_shot_ms * shots, 1)}
        for k, r in res.items():
            line[k + "_ms"] = r["ms"]
            line[k + "_speedup_over_plain"] = round(per_shot_ms * shots / r["ms"], 1)
        print(json.dumps(line), flush=True)


def serving_bench(n_requests: int, loads=(0.8,), max_active: int = 4,
                  qubits=(8, 24), shots=(100, 100_000)):
    """Serving workload: the seeded Poisson stream of random noisy U3+CX
    circuits (qubits U{8..24}, depth U{10..60}, shots log-uniform in
    [100, 1e5], depolarizing 1e-3 / 1e-2, complex64), its first n_requests;
    `qubits` and `shots` narrow the ranges (a lighter stream of many more
    requests, for latency percentiles over hundreds of requests).
    First all requests at once (closed loop: capacity), then the same
    requests with Poisson arrivals at each `load` x that capacity (latency).
    `value` is the throughput at the first load."""
    import workloads as W
    import paper_2308_03399_amd.serving as SV

    def requests(rate):
        stream = W.serving_stream(n_requests, rate, seed=0, qubit_range=tuple(qubits),
                                  shots_range=tuple(shots))
        reqs = [SV.Request(circuit=r["circuit"], noise=r["noise"], shots=r["shots"],
                           seed=r["seed"], dtype=r["dtype"], mode="batch", id=r["id"])
                for r in stream]
        return reqs, [r["arrival_s"] for r in stream]

    def log(tag, rep):
        for res in rep["results"]:
            print(f"[serve {tag}] request {res.id}: {res.shots} shots, "
                  f"{len(res.chunks)} chunks, latency {res.latency:.3f} s",
                  file=sys.stderr, flush=True)

    def summary(rep):
        return {"makespan_s": round(rep["makespan_s"], 3),
                "shots_gates_per_s": rep["shots_gates_per_s"],
                "requests_per_s": round(rep["requests_per_s"], 4),
                "p50_latency_s": round(rep["p50_s"], 4),
                "p99_latency_s": round(rep["p99_s"], 4),
                "mean_latency_s": round(rep["mean_s"], 4),
                "peak_arena_bytes": rep["peak_bytes"]}

    reqs, _ = requests(1.0)
    # warm-up: first request only (library load, kernel modules)
    with SV.Server(max_active=max_active) as srv:
        srv.submit(SV.Request(circuit=reqs[0].circuit, noise=reqs[0].noise,
                              shots=min(reqs[0].shots, 256), seed=0)).wait()
    with SV.Server(max_active=max_active) as srv:
        closed = SV.replay(srv, reqs, [0.0] * len(reqs))
    log("closed", closed)
    cap = closed["requests_per_s"]
    poisson = {}
    first = None
    for load in loads:
        reqs, arrivals = requests(load * cap)
        with SV.Server(max_active=max_active) as srv:
            rep = SV.replay(srv, reqs, arrivals)
        log(f"poisson {load}", rep)
        poisson[str(load)] = dict(summary(rep), arrival_rate_per_s=round(load * cap, 5))
        if first is None:
            first = rep
    out = {
        "metric": "serving: shots×gates/s with p50/p99 latency, Poisson stream of noisy circuits",
        "value": first["shots_gates_per_s"],
        "unit": "shots*gates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": first["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": f"c5_serving: first {n_requests} requests of the seed-0 Poisson "
                        f"stream; qubits U{{{qubits[0]}..{qubits[1]}}}, depth U{{10..60}}, "
                        f"shots log-uniform [{shots[0]}, {shots[1]}]; depolarizing "
                        "1e-3 / 1e-2; batch mode",
            "requests": [{"id": r.id, "qubits": r.n_qubits, "shots": r.shots,
                          "gates": r.gates, "latency_s": round(r.latency, 4),
                          "chunks": len(r.chunks)} for r in first["results"]],
            "total_shots_gates": sum(r.shots * r.gates for r in first["results"]),
            "max_active": max_active,
            "loads": list(loads),
        },
        "serving": {"poisson": poisson, "closed_loop": summary(closed)},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c3_20q", choices=sorted(WORKLOADS),
                    help="c3_20q: the headline (default); c4_26q: 26 qubits x 80 layers U3+CZ, "
                         "2000 shots in one launch")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--dtype", default=None, choices=["c64", "c128"])
    ap.add_argument("--mode", default="batch", choices=["batch", "branch"])
    ap.add_argument("--shots-per-step", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c128", action="store_true",
                    help="skip the complex128 wave reported beside the c64 value")
    ap.add_argument("--no-branch", action="store_true",
                    help="skip the shot-branching wave reported beside the batch value")
    ap.add_argument("--plain-shots", type=int, default=None,
                    help="shots of the plain per-shot FP64 form timed for the speedup (0: skip)")
    ap.add_argument("--qft", type=str, default="",
                    help="instead of the headline workload: the paper's QFT comparison, "
                         "comma-separated qubit counts (4000 shots, 1%% noise)")
    ap.add_argument("--serve", type=int, default=0,
                    help="instead of the headline workload: the serving stream, this many "
                         "requests (closed loop, then Poisson at --serve-loads x its capacity)")
    ap.add_argument("--serve-loads", type=str, default="0.8",
                    help="comma-separated offered loads, as fractions of the closed-loop capacity")
    ap.add_argument("--serve-qubits", type=str, default="8,24",
                    help="qubit range of the serving stream (default: the workload's 8,24)")
    ap.add_argument("--serve-shots", type=str, default="100,100000",
                    help="shot range of the serving stream (default: the workload's 100,100000)")
    ap.add_argument("--error-sweep", type=str, default="",
                    help="instead of the headline workload: the paper's error-ratio experiment "
                         "(QFT, 4000 shots), comma-separated qubit counts")
    ap.add_argument("--error-probs", type=str, default="1e-4,1e-3,1e-2,5e-2")
    ap.add_argument("--one-launch", type=int, default=0,
                    help="for profilers: one sv_run_circuit of this many shots of --workload, "
                         "its stats as one JSON line")
    ap.add_argument("--tile-qubits", type=int, default=0)
    ap.add_argument("--graph", action="store_true",
                    help="replay each step's launches from the handle's HIP graph")
    ap.add_argument("--copy-calibrate", type=int, default=0,
                    help="for counter calibration: a device copy of this many MiB, 3 times")
    args = ap.parse_args()
    spec = WORKLOADS[args.workload]
    args.dtype_given = args.dtype
    for k in ("steps", "warmup", "shots_per_step", "plain_shots", "dtype"):
        if getattr(args, k) is None:
            setattr(args, k, spec[k])
    if args.workload == "c4_26q":
        # 26-qubit states: no FP64 wave at full width (1 GiB per state), no
        # branch wave (fewer slots than shots), no oracle timing (one shot
        # is ~10 min of host time)
        args.no_c128 = args.no_branch = args.no_cpu_baseline = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: shots would shard across GPUs "
              "by shot-id range with no exchange, and the library launches "
              "on one device; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2308_03399_amd import Simulator

    if args.copy_calibrate:
        copy_calibrate(args.copy_calibrate)
        return
    if args.one_launch:
        args.dtype = getattr(args, "dtype_given", None)
        one_launch(args)
        return
    if args.error_sweep:
        error_ratio_sweep([int(x) for x in args.error_sweep.split(",")],
                          [float(x) for x in args.error_probs.split(",")])
        return
    if args.serve:
        serving_bench(args.serve, tuple(float(x) for x in args.serve_loads.split(",")),
                      qubits=[int(x) for x in args.serve_qubits.split(",")],
                      shots=[int(x) for x in args.serve_shots.split(",")])
        return
    if args.qft:
        for n in [int(x) for x in args.qft.split(",")]:
            qft_comparison(n)
        return

    w = W.workload(args.workload)
    circ, noise, seed = w["circuit"], w["noise"], w["seed"]
    gates = W.count_gates(circ)
    B = args.shots_per_step
    sim = Simulator(circ["n_qubits"], B, dtype=args.dtype, mode=args.mode,
                    **({"graph": 1} if args.graph else {}))
    stream = sim.stream

    def step(idx):
        sim_opts_offset = (idx % max(1, (w["shots"] // B))) * B
        from paper_2308_03399_amd import sv_batch_set_option
        sv_batch_set_option(sim.h, "shot_offset", sim_opts_offset)
        sim.run(circ, noise, seed=seed)
        counts = sim.counts(capacity=B)
        return sim.stats(), counts

    mem_first = None  # per-shot registers of shot ids 0..B-1 (untimed warm-up)
    for i in range(args.warmup):
        step(i)
        progress(f"warm-up step {i + 1}/{args.warmup} done")
        if i == 0:
            mem_first = sim.memory()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        st, counts = step(i)
        assert sum(counts.values()) == B
        stats.append(st)
        progress(f"timed step {i + 1}/{args.steps}: {st['exec_ms']:.1f} ms executor")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    total_shots = B * args.steps
    value = total_shots * gates / dt
    exec_ms = sum(s["exec_ms"] for s in stats)
    launches = sum(s["exec_launches"] for s in stats)
    amp_bytes = sum(s["amp_bytes"] for s in stats)
    flops = sum(s["flops"] for s in stats)
    gbs = amp_bytes / (exec_ms * 1e-3) / 1e9
    tfs = flops / (exec_ms * 1e-3) / 1e12
    alu_peak = FP32_VECTOR_PEAK_TF if args.dtype == "c64" else FP64_VECTOR_PEAK_TF
    frac_hbm = gbs / HBM_PEAK_GBS
    frac_alu = tfs / alu_peak
    traffic = measured_traffic(args.workload, args.dtype, B, args.mode,
                               int(amp_bytes / max(launches, 1)))
    if frac_hbm >= frac_alu:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(frac_hbm, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tfs, 3), "peak": alu_peak,
                "unit": "TFLOP/s", "frac": round(frac_alu, 4)}
    roof["traffic"] = traffic
    roof["kernel"] = "svb::exec_kernel_mfma" if stats[0]["mfma"] else "svb::exec_kernel"
    roof["launch_ms"] = round(exec_ms / max(launches, 1), 3)
    roof["algorithmic_bytes_per_launch"] = int(amp_bytes / max(launches, 1))
    roof["algorithmic_flops_per_launch"] = int(flops / max(launches, 1))
    roof["hbm_gbs"] = round(gbs, 1)
    roof["hbm_frac"] = round(frac_hbm, 4)
    roof["alu_tflops"] = round(tfs, 3)
    roof["alu_frac"] = round(frac_alu, 4)

    out = {
        "metric": spec["metric"],
        "value": value,
        "unit": "shots*gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": spec["describe"],
            "shots_per_step": B,
            "total_shots": total_shots,
            "gates_per_shot": gates,
            "mode": args.mode,
            "tile_qubits": stats[0]["tile_qubits"],
            "workers": stats[0]["workers"],
            "passes_per_shot": round(sum(s["passes"] for s in stats) / total_shots, 2),
            "graph_replays": sum(s["graph_replays"] for s in stats),
            "program_uploads": sum(s["program_uploads"] for s in stats),
            "one_qubit_form": "matrix cores" if stats[0]["mfma"] else "vector ALU",
        },
        "roofline": roof,
    }
    sim.close()
    copy_gbs = copy_ceiling_gbs()
    roof["copy_ceiling_gbs"] = round(copy_gbs, 1)
    roof["hbm_frac_of_copy"] = round(gbs / copy_gbs, 4)
    mem128 = None
    progress(f"copy ceiling {copy_gbs:.0f} GB/s")
    if not args.no_c128 and args.dtype == "c64":
        progress("complex128 wave and the complex64 comparison")
        out["c128"], mem128 = other_form(circ, noise, seed, gates, B, "c128", args.mode,
                                         keep_memory=True)
        if mem_first is not None:
            out["c64_vs_fp64"] = c64_vs_fp64(mem_first, mem128, circ, noise, seed)
    elif args.dtype == "c128":
        mem128 = mem_first
    if not args.no_branch and args.mode == "batch":
        progress("shot-branching wave")
        br = other_form(circ, noise, seed, gates, B, args.dtype, "branch")
        br["note"] = ("shot-branching on the same shot ids: shots share a state until a "
                      "draw splits them")
        out["branch"] = br
    if args.plain_shots > 0:
        progress("plain per-shot FP64 form")
        pl = other_form(circ, noise, seed, gates, args.plain_shots, "c128", "plain")
        pl["note"] = ("plain per-shot FP64 form: one state, one kernel per op, first "
                      f"{args.plain_shots} shot ids; time is linear in shots for this form")
        pl["speedup_of_value"] = round(value / pl["value"], 1)
        out["plain_fp64"] = pl
    if not args.no_cpu_baseline:
        import numpy as np
        progress("FP64 oracle on the host cores")
        rec, ids, omem, omarg = cpu_baseline(circ, noise, gates, seed, w["shots"], B)
        out["cpu_baseline"] = rec
        if mem128 is not None:
            # the oracle's registers against the FP64 GPU path on the same ids
            got = np.asarray(mem128)[ids]
            out["oracle_mismatches"] = int(np.sum(got != omem))
            out["oracle_check"] = {"shot_ids": ids, "oracle_min_margin": float(np.min(omarg)),
                                   "oracle_near_ties": int(np.sum(omarg < 1e-9)),
                                   "fp64_wave_near_ties": out.get("c128", {}).get("near_ties")}
    elif args.workload == "c4_26q":
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
