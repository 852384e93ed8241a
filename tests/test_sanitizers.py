"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the library's host runtime (validation, noise expansion, pass planning,
argument and state checks of the C ABI; device entry points replaced by
stand-ins that report no device) and the FP64 oracle are rebuilt with
-fsanitize=address,undefined and driven by a child process with the
sanitizer runtime preloaded. The child must finish without a sanitizer
report and reproduce, bit for bit, what the normal builds give."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "sanitize"))

import oracle  # noqa: E402
import paper_2308_03399_amd as S  # noqa: E402
from sanitize_cases import circuits  # noqa: E402
from test_planner import _plan  # noqa: E402

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-g", "-O1", "-fPIC"]


def _runtime_lib(out):
    csrc = os.path.join(ROOT, "paper_2308_03399_amd", "csrc")
    objs = []
    for src in (os.path.join(csrc, "runtime.cpp"), os.path.join(HERE, "sanitize", "device_stubs.cpp")):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        subprocess.check_call(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__",
                               "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                               "-c", src, "-o", obj])
        objs.append(obj)
    lib = os.path.join(out, "libsvbatch_sanitized.so")
    subprocess.check_call(["g++", "-shared", "-fsanitize=address,undefined", "-o", lib, *objs,
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    return lib


def _oracle_lib(out):
    lib = os.path.join(out, "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-std=gnu11", *SAN, "-fopenmp", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "traj.c"), "-lm"])
    return lib


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_host_runtime_and_oracle_under_sanitizers(tmp_path):
    out = str(tmp_path)
    rt = _runtime_lib(out)
    orc = _oracle_lib(out)
    cases = circuits()
    exp = {"plans": {}, "invalid": {}, "oracle": {}}
    for name, (circ, noise, tile, regs) in cases["plans"].items():
        exp["plans"][name] = [a.tolist() for a in _plan(circ, noise, tile, regs)]
    for name, (circ, noise) in cases["invalid"].items():
        exp["invalid"][name] = 4 if name == "not_attached" else 1   # SV_ESTATE, SV_EINVAL
    for name, (circ, noise, shots, seed) in cases["oracle"].items():
        mem, marg = oracle.run(circ, noise, shots, seed=seed, want_margins=True)
        exp["oracle"][name] = {"memory": [int(x) for x in mem],
                               "margins": [float(x) for x in np.asarray(marg)]}
    ej = os.path.join(out, "expected.json")
    with open(ej, "w") as f:
        json.dump(exp, f)
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ,
               LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               SVB_SANITIZED_RUNTIME=rt, SVB_SANITIZED_ORACLE=orc, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitize", "drive.py"), ej],
                       env=env, capture_output=True, text=True, timeout=600)
    log = r.stdout + r.stderr
    assert r.returncode == 0, log[-4000:]
    assert "SANITIZED_OK" in r.stdout, log[-4000:]
    assert "AddressSanitizer" not in log and "runtime error:" not in log, log[-4000:]
