"""Benchmark of the FZ-GPU hot path on one MI355X.

A step is one pass of the whole path over one field resident in HBM:
value-range error bound (min/max pass), compression (prequantization,
Lorenzo, 16-bit codes, bitshuffle, zero-block encoder with its prefix sum)
and decompression back to fp32.  The field is the 512^3 cosmology-like
lognormal stand-in (exp of a Gaussian random field with a k^-3 spectrum,
sigma 1.5), relative error bound 1e-3 by default.

Prints one JSON line.  ``value`` is the round-trip throughput over the input
bytes (4N / (t_compress + t_decompress)); the per-direction rates, the
compression ratio, the roofline of the dominant kernel (HIP events on the
stream the kernels run on) and the oracle timed on the host cores are added.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.join(HERE, "tests"))

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, public figure


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=512, help="edge of the cubic lognormal field")
    p.add_argument("--eb", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=300)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum CPU time of the oracle baseline")
    p.add_argument("--calib-copy", action="store_true",
                   help="also run one plain elementwise copy of the field (4N bytes read, 4N written) before the timed "
                        "region: the reference dispatch that scales the HBM counters of a profiling run")
    return p.parse_args()


# kernel sources whose HBM counters profiles/traffic.json records
KERNEL_SOURCES = {
    "k_compress": ["fz_compress.hip", "fz_compress_dev.hpp", "fz_device.hpp", "fz_format.hpp"],
    "k_decompress": ["fz_decompress.hip", "fz_decompress_dev.hpp", "fz_device.hpp", "fz_format.hpp"],
}


def source_digest(kernel):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, "paper_2304_12557_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, dims, eb):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel calibration), or
    None if the kernel's sources changed since, or the workload differs."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != source_digest(kernel):
        return None
    if list(rec.get("dims", [])) != list(dims) or float(rec.get("eb", -1)) != float(eb):
        return None
    return int(rec["hbm_bytes"])


def cpu_baseline(x, eb, min_seconds):
    """The oracle (plain C; OpenMP over chunks for compression, one thread for
    decompression) on the same field, repeated until at least `min_seconds`
    of CPU work; GB/s over input bytes for compress + decompress."""
    import numpy as np
    from oracle import oracle as O

    threads = min(os.cpu_count() or 1, 16)
    tc = td = 0.0
    reps = 0
    while tc + td < min_seconds:
        t0 = time.perf_counter()
        s, st = O.compress(x, eb, O.EB_REL, threads=threads)
        t1 = time.perf_counter()
        _, err = O.decompress(s, x.shape)
        t2 = time.perf_counter()
        assert st == 0 and err == 0
        tc += t1 - t0
        td += t2 - t1
        reps += 1
    return {
        "value": round(reps * x.nbytes / 1e9 / (tc + td), 4),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "the whole %dx%dx%d field, %d x (compress with %d OpenMP threads + single-thread decompress); "
                  "compress %.3f s, decompress %.3f s per pass" % (
                      x.shape[0], x.shape[1], x.shape[2], reps, threads, tc / reps, td / reps),
    }


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (each field is compressed on "
              "the GPU that holds it); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2304_12557_amd as fz
    import synth

    dev = torch.device("cuda:0")
    x = synth.lognormal3d(seed=a.seed, n=a.n)
    shape = x.shape
    N = x.size
    in_bytes = 4 * N
    xt = torch.from_numpy(x).to(dev)
    buf = torch.empty(fz.compress_bound(shape), dtype=torch.uint8, device=dev)
    y = torch.empty(shape, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        fz.compress(xt, a.eb, "rel", out=buf)
        fz.decompress(buf, shape, out=y)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    if a.calib_copy:
        ycopy = torch.empty_like(xt)
        torch.neg(xt, out=ycopy)  # an elementwise kernel of its own name: 4N bytes in, 4N out
        torch.cuda.synchronize()
        del ycopy
    info = fz.stream_info(buf)
    assert info["status"] == 0
    s_bytes = int(info["total_bytes"])

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        ev[k][0].record(stream)
        fz.compress(xt, a.eb, "rel", out=buf)
        ev[k][1].record(stream)
        fz.decompress(buf, shape, out=y)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    tc = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))  # ms, REL compress (min/max + params + main)
    td = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))

    # the main compression kernel alone: the same stream in ABS mode with the
    # absolute bound the relative one produced (skips the min/max pass)
    eb_abs = a.eb * (float(info["vmax"]) - float(info["vmin"]))
    abs_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(a.steps)]
    for k in range(a.steps):
        abs_ev[k][0].record(stream)
        fz.compress(xt, eb_abs, "abs", out=buf)
        abs_ev[k][1].record(stream)
    torch.cuda.synchronize()
    tca = float(np.mean([e[0].elapsed_time(e[1]) for e in abs_ev]))

    # roofline of the dominant kernel: the decompression kernel, the longest
    # single kernel of the step, and the only one fz_decompress launches
    # (without an error word), so the events on its stream bracket exactly it.
    # Algorithmic bytes: the stream read plus the fp32 output written.
    name, alg, t_ms = "k_decompress", in_bytes + s_bytes, td
    achieved = alg / (t_ms * 1e-3) / 1e9
    out = {
        "metric": "compress/decompress GB/s (input bytes, % HBM peak) + ratio; batched p50/p99",
        "value": round(in_bytes / 1e9 / ((tc + td) * 1e-3), 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lognormal3d %d^3 fp32 (cosmology-like), REL eb %g, compress + decompress"
                               % (a.n, a.eb), "dims": list(shape), "eb": a.eb, "eb_mode": "rel"},
        "compress_GBps": round(in_bytes / 1e9 / (tc * 1e-3), 2),
        "compress_abs_GBps": round(in_bytes / 1e9 / (tca * 1e-3), 2),
        "decompress_GBps": round(in_bytes / 1e9 / (td * 1e-3), 2),
        "compress_pct_hbm": round(100 * in_bytes / 1e9 / (tc * 1e-3) / HBM_PEAK_GBPS, 2),
        "decompress_pct_hbm": round(100 * in_bytes / 1e9 / (td * 1e-3) / HBM_PEAK_GBPS, 2),
        "ratio": round(in_bytes / s_bytes, 3),
        "stream_bytes": s_bytes,
        "roofline": {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(name, shape, a.eb),
                     "algorithmic_bytes": int(alg), "avg_launch_ms": round(t_ms, 4)},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, a.eb, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
