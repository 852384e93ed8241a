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


def test_autotune_probes_the_one_qubit_form_for_complex64(tmp_path):
    circ = W.random_layered(16, 4, seed=6, two_qubit="cz")
    noise = W.depol_model(gates2=("cz",))
    cache = str(tmp_path / "tune64.json")
    say("case autotune 16q c64 with the one-qubit form")
    res = AT.tune(circ, noise, dtype="c64", waves=1, cache_path=cache, verbose=True)
    forms = {p["mfma"] for p in res["probes"] if "mfma" in p["options"]}
    assert forms == {0, 1}  # vector ALU and matrix cores both probed
    assert res["ms_per_shot"] == min(p["ms_per_shot"] for p in res["probes"])
    shots = 128
    got = gpu_run(circ, noise, shots, dtype="c64", seed=4, **res["options"])
    assert got["stats"]["mfma"] == res["mfma"]
    assert mismatches(got["memory"], oracle_memory(circ, noise, shots, seed=4)) <= 1
