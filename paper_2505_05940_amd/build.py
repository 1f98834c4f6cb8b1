"""Builds libmodal.so in-tree for gfx950 with hipcc.

    python -m paper_2505_05940_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmodal.so")

ARCH = os.environ.get("MODAL_OFFLOAD_ARCH", "gfx950")

# Device code: no FP contraction except explicit fmaf (the float-float
# arithmetic depends on it) and no packed-FP32 instructions.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {os.path.basename(cmd[-1])}")
    return r


def build(verbose: bool = False) -> str:
    """Compiles every source of the library; returns the path of the .so."""
    hipcc = _hipcc()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = [("step_kernel.hip", True), ("grad_kernel.hip", True), ("shared_kernel.hip", True),
            ("linear_kernel.hip", True), ("tf_kernel.hip", True), ("chip_kernel.hip", True),
            ("modal_api.cpp", True),
            ("mlp_kernels.hip", True), ("mlp_api.cpp", True), ("coupling_host.cpp", False)]

    def compile_one(item):
        src, hip = item
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        path = os.path.join(CSRC, src)
        if hip:
            cmd = [hipcc, *HIP_FLAGS, "-x", "hip", "-c", "-o", obj, path]
        else:
            cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-pthread",
                   "-I", os.path.join(ROOT, "include"), "-c", "-o", obj, path]
        r = _run(cmd)
        if verbose and (r.stdout or r.stderr):
            sys.stderr.write(r.stdout + r.stderr)
        return obj

    # the translation units compile independently (at most 8 at a time)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
