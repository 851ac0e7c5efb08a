"""Compile the gfx950 library ``libmi355gemm.so`` in-tree with hipcc.

Every source under ``csrc/`` (HIP kernels and the C++ host runtime) is
compiled for gfx950 only and linked into one shared library that exports the
C-ABI declared in ``include/mi355gemm.h``.  The compiler's per-kernel
resource report (registers, scratch, occupancy, LDS) is kept in
``_build/kernel_resources.txt``; a kernel that spills registers to scratch
memory fails the build, since every tile is sized to fit its register budget.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmi355gemm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-I", os.path.join(ROOT, "include"),
    # packed FP32 instructions stay out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


_REMARK = re.compile(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]|VGPRs|AGPRs|VGPRs Spill|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s+(\S+)")


def _resources(stderr: str) -> list:
    """(kernel, {field: value}) from the kernel-resource-usage remarks."""
    out = []
    for ln in stderr.splitlines():
        m = _REMARK.search(ln)
        if not m:
            continue
        if m.group(1) == "Function Name":
            out.append((m.group(2), {}))
        elif out:
            out[-1][1][m.group(1)] = m.group(2)
    return out


def _compile(src: str, verbose: bool):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    warn = [ln for ln in r.stderr.splitlines() if "warning" in ln and "packed-fp32-ops" not in ln]
    if warn and verbose:
        print("\n".join(warn), file=sys.stderr)
    return obj, _resources(r.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = list(ex.map(lambda s: _compile(s, verbose), srcs))
    objs = [o for o, _ in done]
    kernels = sorted({k: v for _, res in done for k, v in res}.items())
    with open(os.path.join(BUILD, "kernel_resources.txt"), "w") as f:
        for k, v in kernels:
            f.write(k + "  " + "  ".join(f"{a}={b}" for a, b in sorted(v.items())) + "\n")
    spills = [k for k, v in kernels
              if v.get("ScratchSize [bytes/lane]", "0") != "0" or v.get("VGPRs Spill", "0") != "0"]
    if spills:
        raise RuntimeError("kernels spill registers to scratch memory: " + ", ".join(spills))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
