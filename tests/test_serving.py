"""Host logic of the serving loop (no GPU): chunk assembly over global shot
ids, the HBM budget, slot concurrency, admission errors. A fake backend
stands in for the device and returns a fixed function of (seed, shot id),
so any gap, overlap or misplaced chunk shows in the per-shot results."""
import threading
import time

import numpy as np
import pytest

from paper_2308_03399_amd import serving as SV


def _expected(seed, lo, hi):
    ids = np.arange(lo, hi, dtype=np.uint64)
    return (ids * np.uint64(2654435761) + np.uint64(seed)) & np.uint64(0xFFFFF)


class FakeBackend:
    def __init__(self, capacity=8, free=10_000, per_state=10, base=5, sleep=0.002):
        self._cap, self._free = capacity, free
        self.per_state, self.base, self.sleep = per_state, base, sleep
        self.lock = threading.Lock()
        self.live_bytes = 0
        self.max_live_bytes = 0
        self.live_chunks = 0
        self.max_live_chunks = 0
        self.calls = []

    def capacity(self):
        return self._cap

    def free_bytes(self):
        return self._free

    def make_stream(self):
        return None

    def prepare(self, req):
        return ("prepared", req.id)

    def footprint(self, req, n_shots, workers):
        return self.base + self.per_state * workers

    def run(self, req, prepared, offset, n_shots, workers, arena_bytes, stream):
        assert prepared == ("prepared", req.id)
        assert arena_bytes == self.footprint(req, n_shots, workers)
        assert 1 <= workers <= n_shots
        with self.lock:
            self.live_bytes += arena_bytes
            self.live_chunks += 1
            self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
            self.max_live_chunks = max(self.max_live_chunks, self.live_chunks)
            self.calls.append((req.id, offset, n_shots, workers))
        time.sleep(self.sleep * -(-n_shots // workers))
        with self.lock:
            self.live_bytes -= arena_bytes
            self.live_chunks -= 1
        mem = _expected(req.seed, offset, offset + n_shots)
        keys, cnt = np.unique(mem, return_counts=True)
        return mem, {int(k): int(c) for k, c in zip(keys, cnt)}


def _req(i, shots, n=10, seed=None):
    circ = {"n_qubits": n, "n_clbits": n,
            "ops": [{"kind": "u3", "qubits": [0], "params": [0.1, 0.2, 0.3]}] * 5}
    return SV.Request(circuit=circ, noise=None, shots=shots,
                      seed=i * 7 + 1 if seed is None else seed, id=i)


def test_chunks_cover_every_shot_once():
    fb = FakeBackend(capacity=4)
    with SV.Server(max_active=3, hbm_bytes=10_000, chunk_ms=0.5, backend=fb) as s:
        reqs = [_req(i, shots) for i, shots in enumerate([1, 7, 64, 300, 33])]
        tickets = [s.submit(r) for r in reqs]
        results = [t.wait(60) for t in tickets]
    for r, res in zip(reqs, results):
        assert np.array_equal(res.memory, _expected(r.seed, 0, r.shots))
        # chunks tile [0, shots) in order
        pos = 0
        for c in res.chunks:
            assert c.offset == pos and c.shots >= 1
            pos += c.shots
        assert pos == r.shots
        # the merged chunk histograms are the histogram of the whole request
        keys, cnt = np.unique(res.memory, return_counts=True)
        assert res.counts == {int(k): int(c) for k, c in zip(keys, cnt)}
        assert list(res.counts) == sorted(res.counts)
        assert res.gates == 5
        assert res.t_submit <= res.t_start <= res.t_done
    # the 300-shot request ran in several chunks (measured wave time)
    assert len(results[3].chunks) > 1


def test_hbm_budget_is_never_exceeded_and_chunks_overlap():
    fb = FakeBackend(capacity=16, per_state=10, base=5)
    budget = 5 + 10 * 12  # one 12-workgroup chunk, or several smaller ones
    with SV.Server(max_active=4, hbm_bytes=budget, chunk_ms=1.0, backend=fb) as s:
        tickets = [s.submit(_req(i, 200)) for i in range(6)]
        for t in tickets:
            t.wait(60)
        assert s.peak_bytes <= budget
    assert fb.max_live_bytes <= budget
    assert fb.max_live_chunks >= 2
    # shares shrank to fit: no call used more workgroups than the budget holds
    assert max(w for _, _, _, w in fb.calls) <= 12


def test_slots_bound_concurrency():
    fb = FakeBackend(capacity=8, sleep=0.003)
    with SV.Server(max_active=2, hbm_bytes=10_000, chunk_ms=1.0, backend=fb) as s:
        tickets = [s.submit(_req(i, 50)) for i in range(5)]
        for t in tickets:
            t.wait(60)
    assert fb.max_live_chunks <= 2


def test_request_larger_than_budget_fails_alone():
    fb = FakeBackend(per_state=100, base=5)
    with SV.Server(max_active=2, hbm_bytes=50, backend=fb) as s:
        bad = s.submit(_req(0, 10))
        with pytest.raises(MemoryError):
            bad.wait(30)


def test_share_splits_capacity_between_running_requests():
    fb = FakeBackend(capacity=8, sleep=0.004)
    with SV.Server(max_active=2, hbm_bytes=10_000, chunk_ms=2.0, backend=fb) as s:
        a = s.submit(_req(0, 400))
        b = s.submit(_req(1, 400))
        a.wait(60)
        b.wait(60)
    # while both ran, each chunk took at most half of the 8 workgroups
    assert any(w == 4 for _, _, _, w in fb.calls)
    assert max(w for _, _, _, w in fb.calls) <= 8


def test_submit_validation():
    fb = FakeBackend()
    with SV.Server(max_active=1, hbm_bytes=100, backend=fb) as s:
        with pytest.raises(ValueError):
            s.submit(_req(0, 0))
        r = _req(1, 3)
        r.mode = "plain"
        with pytest.raises(ValueError):
            s.submit(r)
    with pytest.raises(RuntimeError):
        s.submit(_req(2, 3))


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert SV.percentile(v, 50) == 50
    assert SV.percentile(v, 99) == 99
    assert SV.percentile(v, 100) == 100
    assert SV.percentile([3.0], 99) == 3.0


def test_replay_reports_latency_and_throughput():
    fb = FakeBackend(capacity=4, sleep=0.001)
    reqs = [_req(i, 20) for i in range(4)]
    with SV.Server(max_active=2, hbm_bytes=10_000, backend=fb) as s:
        rep = SV.replay(s, reqs, [0.0, 0.01, 0.02, 0.03])
    assert len(rep["results"]) == 4
    assert rep["p50_s"] <= rep["p99_s"]
    assert rep["makespan_s"] >= 0.03
    assert rep["shots_gates_per_s"] == pytest.approx(4 * 20 * 5 / rep["makespan_s"])


class FailingBackend(FakeBackend):
    def run(self, req, prepared, offset, n_shots, workers, arena_bytes, stream):
        if req.id == 1:
            raise RuntimeError("device executor failed")
        return super().run(req, prepared, offset, n_shots, workers, arena_bytes, stream)


def test_a_failing_request_does_not_stop_the_others():
    fb = FailingBackend(capacity=4)
    with SV.Server(max_active=2, hbm_bytes=10_000, backend=fb) as s:
        tickets = [s.submit(_req(i, 40)) for i in range(4)]
        with pytest.raises(RuntimeError):
            tickets[1].wait(30)
        for i in (0, 2, 3):
            assert np.array_equal(tickets[i].wait(30).memory, _expected(tickets[i].request.seed, 0, 40))
        # every reservation was returned
        assert s._used == 0
