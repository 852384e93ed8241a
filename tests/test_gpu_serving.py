"""Serving on the GPU: requests of mixed qubit counts, shot counts, storage
precisions and modes are served concurrently (chunked launches on several
streams). Each request's per-shot registers must equal those of the same
request run alone in one launch: exactly, since the per-shot arithmetic is
the same in both cases. The FP64 requests are also checked against the
oracle."""
import numpy as np
import pytest

import paper_2308_03399_amd.serving as SV
import workloads as W
from gpu_util import gpu_run, mismatches, oracle_memory, say

pytestmark = pytest.mark.gpu

# (qubits, layers, shots, dtype, mode)
SPECS = [(6, 8, 300, "c64", "batch"), (9, 10, 500, "c64", "batch"),
         (12, 6, 400, "c128", "batch"), (14, 5, 300, "c64", "batch"),
         (15, 4, 256, "c64", "batch"), (10, 12, 900, "c128", "branch"),
         (16, 3, 200, "c64", "batch"), (8, 6, 700, "c64", "branch")]


def _requests():
    out = []
    for i, (n, d, shots, dt, mode) in enumerate(SPECS):
        noise = W.depol_model(p1=5e-3, p2=2e-2, readout=(0.01, 0.02))
        out.append(SV.Request(circuit=W.random_layered(n, d, seed=100 + i), noise=noise,
                              shots=shots, seed=1000 + i, dtype=dt, mode=mode, id=i,
                              options={"spin_limit_ms": 60000}))
    return out


def test_each_result_same_alone_and_in_the_mix():
    reqs = _requests()
    say("case serving mix: %d requests, 4 slots, 64 workgroups" % len(reqs))
    # a small workgroup capacity and short chunks force shared, chunked launches
    with SV.Server(max_active=4, capacity=64, chunk_ms=2.0) as srv:
        tickets = [srv.submit(r) for r in reqs]
        results = [t.wait(300) for t in tickets]
    for r, res in zip(reqs, results):
        say(f"request {r.id}: n={r.circuit['n_qubits']} shots={r.shots} {r.dtype} "
            f"{r.mode} chunks={len(res.chunks)}")
        alone = gpu_run(r.circuit, r.noise, r.shots, dtype=r.dtype, mode=r.mode,
                        seed=r.seed)
        assert mismatches(res.memory, alone["memory"]) == 0
        assert res.counts == {k: v for k, v in alone["counts"].items()}
        if r.dtype == "c128":
            exp = oracle_memory(r.circuit, r.noise, r.shots, seed=r.seed)
            assert mismatches(res.memory, exp) == 0
    # the requests overlapped in time and some ran in several chunks
    spans = sorted((res.t_start, res.t_done) for res in results)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert max(len(res.chunks) for res in results) > 1


def test_poisson_replay_reports_latency():
    reqs = _requests()[:5]
    arrivals = [0.0, 0.002, 0.004, 0.03, 0.05]
    say("case serving replay: 5 requests")
    with SV.Server(max_active=3) as srv:
        rep = SV.replay(srv, reqs, arrivals)
    assert rep["p50_s"] <= rep["p99_s"] <= rep["makespan_s"]
    assert rep["shots_gates_per_s"] > 0
    for r, res in zip(reqs, rep["results"]):
        assert res.memory.shape == (r.shots,)
        assert sum(res.counts.values()) == r.shots


def test_large_request_chunked_at_default_capacity_equals_alone():
    # a 20-qubit request split into chunks over the full device capacity,
    # served beside small requests, gives the same registers as one launch
    big = SV.Request(circuit=W.random_layered(20, 10, seed=300), noise=W.depol_model(),
                     shots=2000, seed=77, id=100)
    small = [SV.Request(circuit=W.random_layered(n, 6, seed=310 + n), noise=W.depol_model(),
                        shots=300, seed=n, id=n) for n in (7, 11, 13)]
    say("case serving: 20-qubit request chunked beside small ones")
    with SV.Server(max_active=4, chunk_ms=40.0) as srv:
        tickets = [srv.submit(big)] + [srv.submit(r) for r in small]
        results = [t.wait(300) for t in tickets]
    assert len(results[0].chunks) > 1
    for r, res in zip([big] + small, results):
        alone = gpu_run(r.circuit, r.noise, r.shots, dtype="c64", seed=r.seed)
        assert mismatches(res.memory, alone["memory"]) == 0
