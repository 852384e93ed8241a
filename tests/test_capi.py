"""CPU-side checks of the C-ABI library: it loads, exports every function the
header declares, and rejects bad input before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2308_03399_amd as S
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "svbatch.h")).read()
    return sorted(set(re.findall(r"^\s*(?:sv_status|const char \*)\s*(sv_\w+)\s*\(",
                                 text, re.M)))


def test_header_declares_expected_calls():
    names = _header_functions()
    for need in ("sv_batch_create", "sv_run_circuit", "sv_sample_counts",
                 "sv_batch_attach", "sv_batch_footprint", "sv_get_memory"):
        assert need in names


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    for name in _header_functions():
        assert hasattr(lib, name), name
    assert set(_header_functions()) == set(S.EXPORTED)


def test_create_rejects_bad_sizes():
    for n, shots, dt in ((0, 10, 0), (31, 10, 0), (5, 0, 0), (5, 10, 7)):
        with pytest.raises(S.SvError) as e:
            S.sv_batch_create(n, shots, dt)
        assert e.value.status == 1


def test_options_validation():
    h = S.sv_batch_create(4, 10, S.SV_C64)
    try:
        with pytest.raises(S.SvError):
            S.sv_batch_set_option(h, "no_such_option", 1)
        with pytest.raises(S.SvError):
            S.sv_batch_set_option(h, "tile_qubits", 3)
        with pytest.raises(S.SvError):
            S.sv_batch_set_option(h, "dump_shot", 10)
        S.sv_batch_set_option(h, "mode", S.SV_MODE_BRANCH)
        S.sv_batch_set_option(h, "tile_qubits", 8)
    finally:
        S.sv_batch_destroy(h)


def _run_unattached(circ, noise, n=3, shots=4):
    h = S.sv_batch_create(n, shots, S.SV_C128)
    try:
        S.sv_run_circuit(h, S.marshal(circ, noise), 0)
    finally:
        S.sv_batch_destroy(h)


@pytest.mark.parametrize("bad", [
    {"kind": "u3", "qubits": [3], "params": [0, 0, 0]},             # qubit out of range
    {"kind": "cx", "qubits": [1, 1]},                                # repeated qubit
    {"kind": "measure", "qubits": [0], "clbits": [64]},              # clbit >= 64
    {"kind": "unitary", "qubits": [0], "matrix": [[1, 1], [0, 1]]},  # not unitary
    {"kind": "x", "qubits": [0], "cond": [1, 2]},                    # value outside mask
    {"kind": "bfunc", "qubits": [0], "clbits": [1], "mask": 1, "value": 1},  # branch op with qubits
    {"kind": "bfunc", "clbits": [64], "mask": 1, "value": 0},       # branch-op clbit >= 64
])
def test_invalid_ops_are_rejected_without_device(bad):
    circ = {"n_qubits": 3, "n_clbits": 1, "ops": [bad]}
    with pytest.raises(S.SvError) as e:
        _run_unattached(circ, None)
    assert e.value.status == 1


def test_invalid_noise_is_rejected():
    circ = {"n_qubits": 3, "n_clbits": 0, "ops": [{"kind": "h", "qubits": [0]}]}
    bad_p = W.noise_model([W.rule(["h"], W.pauli_table([0.5, 0.4], ["I", "X"]))])
    with pytest.raises(S.SvError) as e:
        _run_unattached(circ, bad_p)
    assert e.value.status == 1
    bad_k = W.noise_model([W.rule(["h"], W.kraus_channel([[[1, 0], [0, 0.5]]]))])
    with pytest.raises(S.SvError) as e:
        _run_unattached(circ, bad_k)
    assert e.value.status == 1
    # a rule attaches only to gates of its own width: a 2-qubit channel on a
    # 1-qubit gate kind adds nothing, and the circuit is valid (it then
    # needs an arena, SV_ESTATE)
    wrong_width = W.noise_model([W.rule(["h"], W.depolarizing_pauli(0.1, 2))])
    with pytest.raises(S.SvError) as e:
        _run_unattached(circ, wrong_width)
    assert e.value.status == 4


def test_valid_circuit_needs_arena():
    circ = W.random_layered(3, 2, seed=0)
    with pytest.raises(S.SvError) as e:
        _run_unattached(circ, W.depol_model())
    assert e.value.status == 4  # SV_ESTATE


def test_empty_circuit_is_valid_and_needs_arena():
    # no ops is a valid circuit (every register 0); it still needs the arena
    with pytest.raises(S.SvError) as e:
        _run_unattached({"n_qubits": 3, "n_clbits": 3, "ops": []}, W.depol_model())
    assert e.value.status == 4  # SV_ESTATE, not SV_EINVAL


def test_results_before_run_are_refused():
    h = S.sv_batch_create(3, 4, S.SV_C64)
    try:
        with pytest.raises(S.SvError) as e:
            S.sv_get_memory(h, 4)
        assert e.value.status == 4
        with pytest.raises(S.SvError) as e:
            S.sv_get_stats(h)
        assert e.value.status == 4
    finally:
        S.sv_batch_destroy(h)


def test_large_mid_circuit_measure_is_unsupported():
    circ = {"n_qubits": 6, "n_clbits": 6,
            "ops": [{"kind": "measure", "qubits": [0, 1, 2, 3, 4], "clbits": [0, 1, 2, 3, 4]},
                    {"kind": "h", "qubits": [0]}]}
    with pytest.raises(S.SvError) as e:
        _run_unattached(circ, None, n=6)
    # validation of sizes happens before the arena check
    assert e.value.status == 5


def test_sweep_argument_checks_without_device():
    circ = {"n_qubits": 2, "n_clbits": 0, "ops": [{"kind": "u3", "qubits": [0], "params": [0, 0, 0]}]}
    params = np.zeros((3, 1, 3))
    h = S.sv_batch_create(2, 10, S.SV_C128)
    try:
        with pytest.raises(S.SvError) as e:       # 3 sets do not divide 10 shots
            S.sv_run_sweep(h, S.marshal(circ, None), 0, params)
        assert e.value.status == 1
        S.sv_batch_set_option(h, "mode", S.SV_MODE_BRANCH)
        with pytest.raises(S.SvError) as e:       # sweeps run in batch mode only
            S.sv_run_sweep(h, S.marshal(circ, None), 0, np.zeros((2, 1, 3)))
        assert e.value.status == 5
    finally:
        S.sv_batch_destroy(h)


def test_executor_keeps_two_waves_per_simd():
    """The build records hipcc's resource usage of the executor kernels.
    The instantiations that run two workgroups per compute unit must fit
    two waves per SIMD in the unified register file."""
    import json
    from paper_2308_03399_amd import build as B
    if not os.path.exists(B.RESOURCES):
        pytest.skip("library not built")
    with open(B.RESOURCES) as f:
        res = json.load(f)
    for k in B.TWO_WAVE_KERNELS:
        assert res[k]["Occupancy [waves/SIMD]"] >= 2, (k, res[k])
        assert res[k]["VGPRs"] + res[k].get("AGPRs", 0) <= 256, (k, res[k])


def test_resource_remarks_are_parsed():
    from paper_2308_03399_amd import build as B
    text = ("x.hip:1:1: remark: Function Name: _Zfoo [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     VGPRs: 200 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]\n"
            "x.hip:1:1: remark:     Occupancy [waves/SIMD]: 2 [-Rpass-analysis=kernel-resource-usage]\n")
    r = B.parse_resource_usage(text)
    assert r == {"_Zfoo": {"VGPRs": 200, "AGPRs": 0, "Occupancy [waves/SIMD]": 2}}
