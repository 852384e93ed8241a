"""Builds libsvbatch.so (HIP kernels + host runtime + C ABI) for gfx950,
in-tree, with hipcc."""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libsvbatch.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

SOURCES = ["runtime.cpp", "kernels.hip", "kernels_mfma.hip", "counts.hip", "plain.hip", "noalloc.hip"]
# executor translation units (resource-usage remarks, no VGPR spills into AGPRs)
EXEC_SOURCES = ("kernels.hip", "kernels_mfma.hip")
ARCH = os.environ.get("SVB_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed-FP32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(os.path.dirname(HERE), "include")]
# The executor's register budget is the whole unified register file share
# of two waves per SIMD (256 per lane). A spill into an accumulation
# register would push the total over it and halve the occupancy, so
# spills go to scratch memory instead (outside the tile loop).
EXEC_FLAGS = ["-mllvm", "-amdgpu-spill-vgpr-to-agpr=0",
              "-Rpass-analysis=kernel-resource-usage"]
# executor instantiations that must run two workgroups per compute unit
# (complex64 at 16 and 32 amplitudes per thread, in both one-qubit forms,
# complex128 at 16)
TWO_WAVE_KERNELS = ["_ZN3svb11exec_kernelIfLi32EEEvNS_10ExecParamsE",
                    "_ZN3svb11exec_kernelIfLi16EEEvNS_10ExecParamsE",
                    "_ZN3svb16exec_kernel_mfmaIfLi32EEEvNS_10ExecParamsE",
                    "_ZN3svb16exec_kernel_mfmaIfLi16EEEvNS_10ExecParamsE",
                    "_ZN3svb11exec_kernelIdLi16EEEvNS_10ExecParamsE"]
RESOURCES = os.path.join(OUT_DIR, "kernel_resources.json")


def parse_resource_usage(text: str) -> dict:
    """{kernel symbol: {field: value}} from hipcc's resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z][A-Za-z \[\]/]*?):\s+(-?\d+)", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = int(m.group(2))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(BUILD_DIR, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        objs.append(obj)
        extra = EXEC_FLAGS if src in EXEC_SOURCES else []
        cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
    failed = []
    resources = {}
    for src, p in procs:
        out, _ = p.communicate()
        raw = out.decode(errors="replace")
        if src in EXEC_SOURCES:
            resources.update(parse_resource_usage(raw))
        text = "\n".join(l for l in raw.splitlines()
                         if "packed-fp32-ops" not in l and "remark:" not in l
                         and "Rpass" not in l)
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"--- {src}\n{text}\n")
        raise RuntimeError("hipcc failed: " + ", ".join(s for s, _ in failed))
    low = [k for k in TWO_WAVE_KERNELS
           if resources.get(k, {}).get("Occupancy [waves/SIMD]", 0) < 2]
    if low:
        raise RuntimeError("executor occupancy below two waves per SIMD: " + ", ".join(
            f"{k} {resources.get(k)}" for k in low))
    with open(RESOURCES, "w") as f:
        json.dump({k: v for k, v in resources.items() if "exec_kernel" in k}, f, indent=1)
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC",
                           "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
