"""Builds libhg.so (the HIP kernels and the C ABI) and two microbenchmarks
(bench_alu: ALU issue rates; bench_launch: launch and same-word atomic
costs) in-tree for gfx950.

    python -m paper_2003_05293_amd.build

Every HIP source is compiled with packed FP32 instructions disabled
(-target-feature -packed-fp32-ops): the compiler then never emits packed
FP32 adds, multiplies or FMAs on its own.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhg.so")
MICROBENCH = ("bench_alu", "bench_launch")
SOURCES = ["kernels.hip", "kernels_mx.hip", "kernels_sep.hip", "runtime.hip", "api.hip", "engine.hip"]
ARCH = "gfx950"

# Kernel arguments preloaded into SGPRs (gfx950 loads the first 16 dwords
# with the wave; the code object keeps a prologue for firmware without the
# feature): every kernel starts one memory round trip earlier.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libhg)")


def build(verbose: bool = False) -> str:
    """Compile every source and link libhg.so; returns its path."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="hg_build_") as tmp:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [cc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        for cmd, proc in procs:
            if proc.wait() != 0:
                raise subprocess.CalledProcessError(proc.returncode, cmd)
        out_tmp = os.path.join(tmp, "libhg.so")
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        shutil.copyfile(out_tmp, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
        # microbenchmarks behind the roofline and the hand-off design
        # (standalone programs)
        for name in MICROBENCH:
            exe_tmp = os.path.join(tmp, name)
            cmd = [cc, *HIP_FLAGS, os.path.join(CSRC, name + ".hip"), "-o", exe_tmp]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            dst = os.path.join(PKG, name)
            shutil.copyfile(exe_tmp, dst + ".tmp")
            os.chmod(dst + ".tmp", 0o755)
            os.replace(dst + ".tmp", dst)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
