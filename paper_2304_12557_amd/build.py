"""Builds libfzmi.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3, fp contraction off, fp32 denormals kept, packed-fp32 instructions
disabled, and the compiler's wave-level atomic aggregation off (it broadcasts
an atomic's result right after issuing it, so the wave waits for the atomic
there; the compression kernels take their next ticket early and use it a
layer later).  Usage: python -m paper_2304_12557_amd.build  (or build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["fz_api.hip", "fz_compress.hip", "fz_decompress.hip", "fz_batch.hip", "fz_server.hip", "fz_quality.hip", "fz_ablation.hip", "fz_f64.hip", "fz_global.hip", "fz_static.hip"]
LIB = os.path.join(HERE, "libfzmi.so")
ARCH = os.environ.get("FZ_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off", "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function", "-I" + os.path.join(os.path.dirname(HERE), "include"),
]


def build(verbose=False, extra=()):
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for s in SRC:
        o = os.path.join(bdir, s.replace(".hip", ".o"))
        cmd = ["hipcc", "-c", os.path.join(HERE, "csrc", s), "-o", o] + FLAGS + list(extra)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), s))
        objs.append(o)
    for p, s in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode())
            raise RuntimeError("hipcc failed on " + s)
        if verbose and out:
            sys.stderr.write(out.decode())
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
