"""Build libyyg.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: python -m paper_1806_04593_amd.build   (or build() from Python)
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libyyg.so")

SOURCES = ["yyg_kernels.hip", "yyg_kernels_x4.hip", "yyg_batch_sep.hip", "yyg_kernels_sep_lp.hip", "yyg_kernels_lp.hip",
           "yyg_phi_stream.hip", "yyg_noalloc.hip", "yyg_checks.hip", "yyg_tables.cpp", "yyg_host.cpp", "yyg_api.cpp"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in arch VGPRs: without it, loops with few
    # accumulator tiles copy them between VGPRs and AGPRs at every step
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, jobs=None):
    """Compile every source to an object in parallel (one hipcc process per
    source), then link the shared library; replaces LIB atomically."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs, objs = [], []
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1))
    pending = list(SOURCES)
    failed = []
    while pending or procs:
        while pending and len(procs) < jobs:
            src = pending.pop(0)
            obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc] + compile_flags + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd)))
            objs.append(obj)
        src, p = procs.pop(0)
        if p.wait() != 0:
            failed.append(src)
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc ({', '.join(failed)})")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
