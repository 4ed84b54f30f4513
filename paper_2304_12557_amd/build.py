"""Builds libfzmi.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3, fp contraction off, fp32 denormals kept, packed-fp32 instructions
disabled, and the compiler's wave-level atomic aggregation off (it broadcasts
an atomic's result right after issuing it, so the wave waits for the atomic
there; the compression kernels take their next ticket early and use it a
layer later).  The compiler's per-kernel resource report (registers, spills,
LDS, waves per SIMD) is collected from the same compiles into
kernel_resources.json beside the library, for the test that holds the hot
kernels at their occupancy.  Usage: python -m paper_2304_12557_amd.build  (or
build()).
"""
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["fz_api.hip", "fz_compress.hip", "fz_decompress.hip", "fz_batch.hip", "fz_server.hip", "fz_quality.hip", "fz_ablation.hip", "fz_f64.hip", "fz_global.hip", "fz_static.hip"]
LIB = os.path.join(HERE, "libfzmi.so")
RESOURCES = os.path.join(HERE, "kernel_resources.json")
ARCH = os.environ.get("FZ_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off", "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function", "-I" + os.path.join(os.path.dirname(HERE), "include"),
    "-Rpass-analysis=kernel-resource-usage",
]

_FIELDS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch_bytes_per_lane",
           "Occupancy [waves/SIMD]": "waves_per_simd", "VGPRs Spill": "vgpr_spills", "SGPRs Spill": "sgpr_spills",
           "LDS Size [bytes/block]": "lds_bytes"}


def parse_resources(text):
    """Per-kernel figures from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z][^:]*?): (\d+) \[-Rpass-analysis", line)
        if m and cur is not None and m.group(1) in _FIELDS:
            cur[_FIELDS[m.group(1)]] = int(m.group(2))
    return out


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
    resources = {}
    for p, s in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            sys.stderr.write(text)
            raise RuntimeError("hipcc failed on " + s)
        warnings = [ln for ln in text.splitlines() if "warning:" in ln or "error:" in ln]
        if verbose and warnings:
            sys.stderr.write("\n".join(warnings) + "\n")
        resources.update(parse_resources(text))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    with open(RESOURCES, "w") as fh:
        json.dump(resources, fh, indent=1, sort_keys=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
