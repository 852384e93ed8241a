"""Autotuner on the GPU: it probes launch shapes, picks the fastest, caches
the choice, and the chosen shape gives the oracle's per-shot results."""
import json

import pytest

import workloads as W
from paper_2308_03399_amd import autotune as AT
from gpu_util import gpu_run, mismatches, oracle_memory, say

pytestmark = pytest.mark.gpu


def test_autotune_choice_is_cached_and_exact(tmp_path):
    circ = W.random_layered(15, 3, seed=5)
    noise = W.depol_model(p1=5e-3, p2=2e-2,
                          extra_rules=[W.rule(["u3"], W.amplitude_damping_kraus(0.02))])
    cache = str(tmp_path / "tune.json")
    say("case autotune 15q c128")
    res = AT.tune(circ, noise, dtype="c128", waves=1, cache_path=cache, verbose=True)
    assert len(res["probes"]) >= 2
    assert res["ms_per_shot"] == min(p["ms_per_shot"] for p in res["probes"])
    with open(cache) as f:
        assert len(json.load(f)) == 1
    assert AT.tune(circ, noise, dtype="c128", waves=1, cache_path=cache) == res
    shots = 300
    got = gpu_run(circ, noise, shots, dtype="c128", seed=3, **res["options"])
    assert got["stats"]["tile_qubits"] == res["tile_qubits"]
    assert mismatches(got["memory"], oracle_memory(circ, noise, shots, seed=3)) == 0
