"""Autotuner of the executor's launch shape.

The candidates are the choices that change speed but not the method's
result:

* tile qubits k: a streamed pass holds 2^k amplitudes of a state in LDS.
  The register-group width (the gates fused per register sweep) is
  k - 8 qubits, at 2^(k-8) amplitudes per thread.
* tile buffers: 1, with two workgroups per compute unit overlapping, or
  2, where the next tile is fetched while the current one computes.
* workgroups: one or two per compute unit. This sets the number of shots
  each workgroup serves in batch mode.
* complex64 only: the form of the fused one-qubit products (option mfma):
  vector ALU or matrix cores. It is probed on the fastest launch shape.

Every candidate runs a probe of the caller's circuit on a few waves of
shots. The fastest per-shot executor time wins. Results are cached in a
JSON file keyed by the device, the circuit's shape and the noise model's
shape. States that fit one tile (resident in LDS) have a single shape, so
no probe runs for them.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional

from . import Simulator

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "svbatch_autotune.json")


def _resident(n: int, dtype: str) -> bool:
    # at the default tile (13 qubits complex64, 12 complex128) the whole
    # state sits in one workgroup's LDS
    return n <= (12 if dtype == "c128" else 13)


def candidates(n: int, dtype: str, compute_units: int) -> List[Dict]:
    """Launch shapes to probe for an n-qubit state (empty dict: library
    defaults)."""
    if _resident(n, dtype):
        return [{}]
    tiles = [12, 13] if dtype == "c128" else [12, 13, 14]
    out = []
    for k in tiles:
        if k > n:
            continue
        for pipe in (0, 1):
            for per_cu in (1, 2):
                out.append({"tile_qubits": k, "pipeline": pipe,
                            "workers": per_cu * compute_units})
    return out or [{}]


def shape_key(circuit: Dict, noise: Optional[Dict], dtype: str, mode: str,
              device_name: str) -> str:
    """Cache key: what the pass plan and the per-op costs depend on (qubit
    count, op kinds and qubits, noise rule kinds), not the angles."""
    h = hashlib.sha256()
    h.update(f"{device_name}|{dtype}|{mode}|{circuit['n_qubits']}|".encode())
    for op in circuit["ops"]:
        h.update(f"{op['kind']}:{op.get('qubits')};".encode())
    if noise:
        for r in noise.get("rules", []):
            h.update(f"{sorted(r.get('gates', []))}:{r.get('type')}:{r.get('nq')};".encode())
    return h.hexdigest()[:24]


def _probe(circuit, noise, dtype, mode, opts, shots, seed):
    sim = Simulator(circuit["n_qubits"], shots, dtype=dtype, mode=mode, **opts)
    try:
        sim.run(circuit, noise, seed=seed)
        st = sim.stats()
    finally:
        sim.close()
    return st


def tune(circuit: Dict, noise: Optional[Dict], dtype: str = "c64", mode: str = "batch",
         waves: int = 2, seed: int = 0, cache_path: Optional[str] = DEFAULT_CACHE,
         device: str = "cuda:0", verbose: bool = False) -> Dict:
    """Returns {"options": {...}, "ms_per_shot": t, "probes": [...]} for the
    fastest launch shape. `options` go to Simulator / sv_batch_set_option
    as they are."""
    import torch
    props = torch.cuda.get_device_properties(torch.device(device))
    cus = props.multi_processor_count
    key = shape_key(circuit, noise, dtype, mode, props.name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    probes = []
    seen = set()
    best = None
    for opts in candidates(circuit["n_qubits"], dtype, cus):
        shots = waves * int(opts.get("workers", 2 * cus))
        if opts:
            _probe(circuit, noise, dtype, mode, opts, min(shots, 64), seed)  # warm-up
        st = _probe(circuit, noise, dtype, mode, opts, shots, seed)
        shape = (st["tile_qubits"], st["tile_buffers"], st["workers"])
        if shape in seen:  # the library clamped this candidate onto another one
            continue
        seen.add(shape)
        ms = st["exec_ms"] / shots
        rec = {"options": opts, "tile_qubits": st["tile_qubits"],
               "tile_buffers": st["tile_buffers"], "workers": st["workers"],
               "mfma": st["mfma"], "ms_per_shot": ms}
        probes.append(rec)
        if verbose:
            print(f"[autotune] {rec}", flush=True)
        if best is None or ms < best["ms_per_shot"]:
            best = rec
    if dtype == "c64" and not _resident(circuit["n_qubits"], dtype):
        # the one-qubit form on the fastest shape: both explicit choices
        for mf in (1, 2):
            opts = dict(best["options"], mfma=mf)
            shots = waves * int(opts.get("workers", 2 * cus))
            _probe(circuit, noise, dtype, mode, opts, min(shots, 64), seed)  # warm-up
            st = _probe(circuit, noise, dtype, mode, opts, shots, seed)
            ms = st["exec_ms"] / shots
            rec = {"options": opts, "tile_qubits": st["tile_qubits"],
                   "tile_buffers": st["tile_buffers"], "workers": st["workers"],
                   "mfma": st["mfma"], "ms_per_shot": ms}
            probes.append(rec)
            if verbose:
                print(f"[autotune] {rec}", flush=True)
            if ms < best["ms_per_shot"]:
                best = rec
    out = {"options": best["options"], "ms_per_shot": best["ms_per_shot"],
           "tile_qubits": best["tile_qubits"], "tile_buffers": best["tile_buffers"],
           "workers": best["workers"], "mfma": best["mfma"], "probes": probes}
    if cache_path:
        cache[key] = out
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return out
