"""Request loop for serving noisy-circuit sampling jobs on one GPU.

Continuous batching of independent requests (circuit, noise model, shot
count, seed). The multi-shot method of the paper, Sec. III, runs every
request; this module only schedules them.

* Slots. Up to ``max_active`` requests are in service at once. Each has a
  runner thread and a HIP stream of its own, at the default priority. A
  request that arrives while others run is admitted as soon as a slot is
  free, and its launches overlap with theirs on the device.
* Chunks. A request runs as a sequence of executor launches (chunks) over
  consecutive shot ranges, using the library's ``shot_offset``. The random
  draws are keyed by the global shot id, so the per-shot results do not
  depend on the chunking. Chunks are sized to about ``chunk_ms`` of
  estimated device time, and always to at least one wave of workgroups.
  The workgroup share of a chunk is re-decided at each chunk boundary, so a
  long request gives up part of the device to requests that arrive after
  it.
* Admission by HBM footprint. Every chunk reserves its arena bytes (from
  ``sv_batch_footprint``) against a device budget before it allocates. A
  chunk that does not fit shrinks its workgroup count (in batch mode its
  state slots are one per workgroup). At one workgroup it waits until
  memory is released. Waiting chunks are served in arrival order.
* States stay resident. A chunk's states live in its arena from
  initialisation to sampling. Nothing is copied to the host except the
  per-shot classical registers.

Results are per-shot registers (``memory``) and their histogram
(``counts``), with the timestamps that latency figures use.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import (SV_C128, SV_C64, SV_MODE_BATCH, SV_MODE_BRANCH, marshal,
               sv_batch_attach, sv_batch_create, sv_batch_destroy,
               sv_batch_footprint, sv_batch_set_option, sv_get_memory,
               sv_run_circuit, sv_sample_counts)

MODES = {"batch": SV_MODE_BATCH, "branch": SV_MODE_BRANCH}
GATE_KINDS = ("u3", "h", "x", "y", "z", "s", "sdg", "t", "tdg", "id",
              "cx", "cz", "swap", "unitary")

# Device time of one shot on one executor workgroup, per amplitude and per
# gate, at the 20-qubit x 60-layer depolarizing + damping workload on MI355X
# (about 0.42 s per shot per workgroup). Only the size of the first chunk
# of a request depends on it; later chunks use the measured rate.
MS_PER_AMP_GATE = 2.2e-7
MIN_AMPS = 1 << 12


@dataclass
class Request:
    circuit: Dict
    noise: Optional[Dict]
    shots: int
    seed: int = 0
    dtype: str = "c64"
    mode: str = "batch"
    id: int = 0
    options: Dict = field(default_factory=dict)


@dataclass
class Chunk:
    offset: int
    shots: int
    workers: int
    arena_bytes: int
    t_start: float
    t_end: float


@dataclass
class Result:
    id: int
    memory: np.ndarray
    counts: Dict[int, int]
    gates: int
    shots: int
    n_qubits: int
    t_submit: float
    t_start: float
    t_done: float
    chunks: List[Chunk]

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class Ticket:
    """Handle of a submitted request."""

    def __init__(self, request: Request):
        self.request = request
        self.t_submit = time.perf_counter()
        self.result: Optional[Result] = None
        self.error: Optional[BaseException] = None
        self._done = threading.Event()

    def done(self) -> bool:
        return self._done.is_set()

    def wait(self, timeout: Optional[float] = None) -> Result:
        if not self._done.wait(timeout):
            raise TimeoutError(f"request {self.request.id} still running")
        if self.error is not None:
            raise self.error
        return self.result


def count_gates(circuit: Dict) -> int:
    return sum(1 for op in circuit["ops"] if op["kind"] in GATE_KINDS)


class DeviceBackend:
    """Executes chunks through the C ABI on one GPU."""

    def __init__(self, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        props = torch.cuda.get_device_properties(self.device)
        self.compute_units = props.multi_processor_count

    def capacity(self) -> int:
        # two executor workgroups per compute unit (the streamed-tile
        # occupancy); smaller resident states would fit more
        return 2 * self.compute_units

    def free_bytes(self) -> int:
        free, _total = self.torch.cuda.mem_get_info(self.device)
        return int(free)

    def make_stream(self):
        self.torch.cuda.set_device(self.device)
        return self.torch.cuda.Stream(device=self.device)

    def prepare(self, req: Request):
        return marshal(req.circuit, req.noise)

    def _handle(self, req: Request, n_shots: int, workers: int, offset: int):
        h = sv_batch_create(req.circuit["n_qubits"], n_shots,
                            SV_C128 if req.dtype == "c128" else SV_C64)
        try:
            sv_batch_set_option(h, "mode", MODES[req.mode])
            sv_batch_set_option(h, "workers", workers)
            if req.mode == "branch" and "slots" not in req.options:
                # the library's automatic branch budget is half the free
                # device memory; a shared device gets a per-chunk share
                sv_batch_set_option(h, "slots", min(n_shots, 4 * workers))
            sv_batch_set_option(h, "shot_offset", offset)
            for k, v in req.options.items():
                sv_batch_set_option(h, k, int(v))
        except BaseException:
            sv_batch_destroy(h)
            raise
        return h

    def footprint(self, req: Request, n_shots: int, workers: int) -> int:
        h = self._handle(req, n_shots, workers, 0)
        try:
            return int(sv_batch_footprint(h)[0])
        finally:
            sv_batch_destroy(h)

    def run(self, req: Request, prepared, offset: int, n_shots: int, workers: int,
            arena_bytes: int, stream):
        """One chunk: per-shot registers and the chunk's histogram (the
        library's device sort and run-length encoding)."""
        torch = self.torch
        h = self._handle(req, n_shots, workers, offset)
        try:
            with torch.cuda.device(self.device), torch.cuda.stream(stream):
                arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
                sv_batch_attach(h, arena.data_ptr(), arena_bytes, stream.cuda_stream)
                # synchronous on `stream`: returns when the launch has finished
                sv_run_circuit(h, prepared, req.seed)
                mem = sv_get_memory(h, n_shots)
                counts = sv_sample_counts(h, capacity=n_shots)
                del arena
            return mem, counts
        finally:
            sv_batch_destroy(h)


class Server:
    """Continuous-batching request loop (see the module docstring)."""

    def __init__(self, device: str = "cuda:0", max_active: int = 4,
                 hbm_bytes: Optional[int] = None, capacity: Optional[int] = None,
                 chunk_ms: float = 200.0, backend=None):
        if max_active < 1:
            raise ValueError("max_active must be >= 1")
        self.backend = backend if backend is not None else DeviceBackend(device)
        self.capacity = int(capacity or self.backend.capacity())
        self.budget = int(hbm_bytes if hbm_bytes else 0.9 * self.backend.free_bytes())
        self.chunk_ms = float(chunk_ms)
        self.max_active = max_active
        self._cv = threading.Condition()
        self._pending: collections.deque = collections.deque()
        self._running = 0
        self._used = 0
        self._peak_used = 0
        self._fp_cache: Dict = {}
        self._mem_queue: collections.deque = collections.deque()  # chunks waiting for bytes
        self._closed = False
        self._threads = [threading.Thread(target=self._runner, daemon=True,
                                          name=f"sv-runner-{i}")
                         for i in range(max_active)]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------ public
    def submit(self, req: Request) -> Ticket:
        if req.shots < 1:
            raise ValueError("shots must be >= 1")
        if req.mode not in MODES:
            raise ValueError(f"mode {req.mode!r}: serving runs batch or branch mode")
        t = Ticket(req)
        with self._cv:
            if self._closed:
                raise RuntimeError("server is closed")
            self._pending.append(t)
            self._cv.notify_all()
        return t

    @property
    def peak_bytes(self) -> int:
        return self._peak_used

    def close(self):
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ----------------------------------------------------------- runners
    def _runner(self):
        stream = self.backend.make_stream()
        while True:
            with self._cv:
                while not self._pending and not self._closed:
                    self._cv.wait()
                if not self._pending:
                    return
                ticket = self._pending.popleft()
                self._running += 1
            try:
                ticket.result = self._serve(ticket, stream)
            except BaseException as e:  # delivered to the caller by wait()
                ticket.error = e
            finally:
                with self._cv:
                    self._running -= 1
                    self._cv.notify_all()
                ticket._done.set()

    def _share(self) -> int:
        with self._cv:
            return max(1, -(-self.capacity // max(1, self._running)))

    def _reserve(self, req: Request, n_shots: int, workers: int):
        """(workers, bytes) of a chunk once its arena is reserved; shrinks
        the workgroup count to fit, then waits in arrival order."""
        cands = [workers]
        while cands[-1] > 1:
            cands.append(max(1, cands[-1] // 2))
        sizes = [(w, self._footprint(req, n_shots, w)) for w in cands]
        if sizes[-1][1] > self.budget:
            raise MemoryError(f"request {req.id}: one state needs {sizes[-1][1]} bytes, "
                              f"budget {self.budget}")
        token = object()
        with self._cv:
            self._mem_queue.append(token)
            try:
                while True:
                    if self._mem_queue[0] is token:
                        free = self.budget - self._used
                        for w, b in sizes:
                            if b <= free:
                                self._used += b
                                self._peak_used = max(self._peak_used, self._used)
                                return w, b
                    self._cv.wait()
            finally:
                self._mem_queue.remove(token)
                self._cv.notify_all()

    def _footprint(self, req: Request, n_shots: int, workers: int) -> int:
        """Arena bytes of a chunk shape, computed once per shape."""
        key = (req.circuit["n_qubits"], req.dtype, req.mode,
               tuple(sorted(req.options.items())), n_shots, workers)
        b = self._fp_cache.get(key)
        if b is None:
            b = self.backend.footprint(req, n_shots, workers)
            self._fp_cache[key] = b
        return b

    def _release(self, nbytes: int):
        with self._cv:
            self._used -= nbytes
            self._cv.notify_all()

    def _serve(self, ticket: Ticket, stream) -> Result:
        req = ticket.request
        n = req.circuit["n_qubits"]
        gates = count_gates(req.circuit)
        prepared = self.backend.prepare(req)
        mem = np.empty(req.shots, dtype=np.uint64)
        counts: collections.Counter = collections.Counter()
        chunks: List[Chunk] = []
        # ms of one wave (one shot per workgroup); refined from measurements
        wave_ms = MS_PER_AMP_GATE * max(1 << n, MIN_AMPS) * max(gates, 1)
        offset = 0
        t_start = None
        while offset < req.shots:
            left = req.shots - offset
            share = self._share()
            waves = max(1, int(self.chunk_ms / max(wave_ms, 1e-6)))
            c = min(left, share * waves)
            w = min(share, c)
            w, nbytes = self._reserve(req, c, w)
            try:
                t0 = time.perf_counter()
                if t_start is None:
                    t_start = t0
                mem[offset:offset + c], part = self.backend.run(req, prepared, offset, c, w,
                                                                nbytes, stream)
                counts.update(part)
                t1 = time.perf_counter()
            finally:
                self._release(nbytes)
            chunks.append(Chunk(offset, c, w, nbytes, t0, t1))
            wave_ms = 1e3 * (t1 - t0) / math.ceil(c / w)
            offset += c
        # chunks cover disjoint shot ranges: their histograms add up
        return Result(id=req.id, memory=mem,
                      counts={k: counts[k] for k in sorted(counts)},
                      gates=gates, shots=req.shots, n_qubits=n, t_submit=ticket.t_submit,
                      t_start=t_start, t_done=time.perf_counter(), chunks=chunks)


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    i = max(0, min(len(v) - 1, math.ceil(q / 100.0 * len(v)) - 1))
    return v[i]


def replay(server: Server, requests: List[Request], arrivals_s: List[float]) -> Dict:
    """Submits each request at its arrival offset (seconds from the start),
    waits for all, and returns latency and throughput figures."""
    t0 = time.perf_counter()
    tickets = []
    for req, a in zip(requests, arrivals_s):
        dt = t0 + a - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(server.submit(req))
    results = [t.wait() for t in tickets]
    t1 = time.perf_counter()
    lat = [r.latency for r in results]
    work = sum(r.shots * r.gates for r in results)
    return {"results": results,
            "makespan_s": t1 - t0,
            "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "mean_s": sum(lat) / len(lat),
            "shots_gates_per_s": work / (t1 - t0),
            "requests_per_s": len(results) / (t1 - t0),
            "peak_bytes": server.peak_bytes}
