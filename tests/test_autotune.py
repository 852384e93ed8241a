"""Autotuner host logic (no GPU): candidate launch shapes and cache keys."""
import workloads as W
from paper_2308_03399_amd import autotune as AT


def test_resident_states_have_one_shape():
    assert AT.candidates(10, "c64", 256) == [{}]
    assert AT.candidates(13, "c64", 256) == [{}]
    assert AT.candidates(12, "c128", 256) == [{}]


def test_streamed_candidates_cover_tiles_buffers_and_workgroups():
    c = AT.candidates(20, "c64", 256)
    assert {x["tile_qubits"] for x in c} == {12, 13, 14}
    assert {x["pipeline"] for x in c} == {0, 1}
    assert {x["workers"] for x in c} == {256, 512}
    assert len(c) == 12
    c = AT.candidates(20, "c128", 256)
    assert {x["tile_qubits"] for x in c} == {12, 13}
    # a tile never exceeds the state
    assert all(x["tile_qubits"] <= 13 for x in AT.candidates(13, "c128", 8))


def test_shape_key_ignores_angles_but_not_structure():
    a = W.random_layered(16, 3, seed=1)
    b = W.random_layered(16, 3, seed=1)
    for op in b["ops"]:
        if op["kind"] == "u3":
            op["params"] = [p + 0.5 for p in op["params"]]
    nm = W.depol_model()
    assert AT.shape_key(a, nm, "c64", "batch", "dev") == AT.shape_key(b, nm, "c64", "batch", "dev")
    c = W.random_layered(16, 3, seed=2)  # other pairings
    assert AT.shape_key(a, nm, "c64", "batch", "dev") != AT.shape_key(c, nm, "c64", "batch", "dev")
    assert AT.shape_key(a, nm, "c64", "batch", "dev") != AT.shape_key(a, nm, "c128", "batch", "dev")
    assert AT.shape_key(a, nm, "c64", "batch", "dev") != AT.shape_key(a, None, "c64", "batch", "dev")
