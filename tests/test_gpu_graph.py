"""Runs replayed from the handle's HIP graph (option graph=1: the
initialisation kernel and the persistent executor as two graph nodes whose
arguments are updated per run) give the same per-shot registers as direct
launches, run after run: different seeds, shot offsets and circuits on one
handle, eager runs of other handles in between, batch and branch mode (with
waiting-list relaunches outside the graph), resident and streamed states."""
import numpy as np
import pytest

import paper_2308_03399_amd as S
import workloads as W
from gpu_util import gpu_run, say

pytestmark = pytest.mark.gpu


def _noise():
    return W.noise_model(
        [W.rule(["u3"], W.depolarizing_pauli(0.05, 1)),
         W.rule(["u3"], W.amplitude_damping_kraus(0.05)),
         W.rule(["cx"], W.depolarizing_pauli(0.1, 2))],
        readout=(0.02, 0.02))


@pytest.mark.parametrize("n,dtype,mode,tile,slots", [
    (6, "c128", "batch", 0, 0), (11, "c128", "batch", 0, 0), (14, "c64", "batch", 12, 0),
    (14, "c128", "branch", 12, 0), (7, "c128", "branch", 0, 3)])
def test_graph_replays_equal_direct_launches(n, dtype, mode, tile, slots):
    noise = _noise()
    shots = 200
    opts = {"tile_qubits": tile} if tile else {}
    if slots:
        opts["slots"] = slots  # few slots: waiting-list relaunches after the graph
    circs = [W.random_layered(n, 4, seed=n), W.random_layered(n, 3, seed=n + 1)]
    sim = S.Simulator(n, shots, dtype=dtype, mode=mode, graph=1, spin_limit_ms=60000, **opts)
    try:
        runs = [(0, 11, 0), (0, 12, 500), (0, 12, 500), (1, 13, 7), (1, 13, 7), (0, 14, 3)]
        prev = None
        for i, (ci, seed, off) in enumerate(runs):
            circ = circs[ci]
            S.sv_batch_set_option(sim.h, "shot_offset", off)
            sim.run(circ, noise, seed=seed)
            got = sim.memory()
            st = sim.stats()
            say(f"case graph n={n} {dtype} {mode} run {i}: circuit {ci} seed {seed} offset {off}, "
                f"replay {st['graph_replays']} upload {st['program_uploads']} "
                f"restarts {st['restarts']}")
            assert st["graph_replays"] == 1
            # the program is uploaded only when it changed
            assert st["program_uploads"] == (0 if prev == ci else 1)
            prev = ci
            exp = gpu_run(circ, noise, shots, dtype=dtype, mode=mode, seed=seed,
                          shot_offset=off, **opts)["memory"]
            assert np.array_equal(got, exp)
        if slots:
            assert st["restarts"] > 0
    finally:
        sim.close()
