"""Child process of tests/test_sanitizers.py, run with the AddressSanitizer
runtime preloaded: drives the sanitized host runtime (planner, validation,
argument and state checks of the C ABI) and the sanitized oracle, and checks
their results against the values the parent computed with the normal
builds."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import paper_2308_03399_amd as S  # noqa: E402
import workloads as W  # noqa: E402

S.LIB_PATH = os.environ["SVB_SANITIZED_RUNTIME"]
oracle._LIB_PATH = os.environ["SVB_SANITIZED_ORACLE"]
expected = json.load(open(sys.argv[1]))
with open("/proc/self/maps") as fh:
    assert "libasan" in fh.read(), "the AddressSanitizer runtime is not loaded"

from test_planner import _plan  # noqa: E402
from sanitize_cases import circuits  # noqa: E402

cases = circuits()
# planner: the same plan as the normal build
for name, (circ, noise, tile, regs) in cases["plans"].items():
    order, opass, ogrp, pmask, gw = _plan(circ, noise, tile, regs)
    got = [order.tolist(), opass.tolist(), ogrp.tolist(), pmask.tolist(), gw.tolist()]
    assert got == expected["plans"][name], f"plan {name} differs"
    print(f"plan {name}: {len(order)} ops, {len(pmask)} passes", flush=True)

# validation and state errors of the C ABI (no device is touched)
for name, (circ, noise) in cases["invalid"].items():
    h = S.sv_batch_create(circ["n_qubits"], 8, S.SV_C64)
    try:
        try:
            S.sv_run_circuit(h, S.marshal(circ, noise), 0)
            raise AssertionError(f"{name}: accepted")
        except S.SvError as e:
            assert e.status == expected["invalid"][name], (name, e.status, str(e))
    finally:
        S.sv_batch_destroy(h)
    print(f"invalid {name}: status {expected['invalid'][name]}", flush=True)
for n, shots, dt in [(0, 1, 0), (31, 1, 0), (4, 0, 0), (4, 1, 7)]:
    try:
        S.sv_batch_create(n, shots, dt)
        raise AssertionError("bad sizes accepted")
    except S.SvError as e:
        assert e.status == 1
h = S.sv_batch_create(3, 4, S.SV_C64)
for key, val in [("no_such_option", 1), ("tile_qubits", 3), ("dump_shot", 4), ("mode", 9)]:
    try:
        S.sv_batch_set_option(h, key, val)
        raise AssertionError(f"option {key}={val} accepted")
    except S.SvError as e:
        assert e.status == 1
for f in (lambda: S.sv_get_memory(h, 4), lambda: S.sv_get_stats(h), lambda: S.sv_sample_counts(h, 4)):
    try:
        f()
        raise AssertionError("results before a run")
    except S.SvError as e:
        assert e.status == 4
S.sv_batch_destroy(h)

# oracle: the same registers and margins as the normal build
for name, (circ, noise, shots, seed) in cases["oracle"].items():
    mem, marg = oracle.run(circ, noise, shots, seed=seed, want_margins=True)
    assert [int(x) for x in mem] == expected["oracle"][name]["memory"], name
    assert np.array_equal(np.asarray(marg), np.asarray(expected["oracle"][name]["margins"])), name
    print(f"oracle {name}: {shots} shots equal", flush=True)
print("SANITIZED_OK", flush=True)
