"""Benchmark of the FZ-GPU hot path on one MI355X.

A step is one pass of the whole path over one field resident in HBM:
value-range error bound (min/max pass), compression (prequantization,
Lorenzo, 16-bit codes, bitshuffle, zero-block encoder with its prefix sum)
and decompression back to fp32.  The field is the 512^3 cosmology-like
lognormal stand-in (exp of a Gaussian random field with a k^-3 spectrum,
sigma 1.5), relative error bound 1e-3 by default.

Prints one JSON line.  ``value`` is the round-trip throughput over the input
bytes (4N / (t_compress + t_decompress)); the per-direction rates, the
compression ratio, every kernel's rate against the HBM roofline with the
dominant one as the headline entry (HIP events on the stream the kernels run
on, the compression's inner points recorded by fz_compress_timed), the
paper-shaped fields, and the oracle timed on the host cores are added.  Each
timed call starts with cold caches (a 1 GiB read in between, outside the
events).
"""
import argparse
import ctypes
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
    p.add_argument("--workload", default="lognormal3d",
                   choices=("lognormal3d", "sine3d", "climate2d", "hurricane3d"),
                   help="the field of the timed steps: the 512^3 cosmology-like lognormal field (default, edge --n), "
                        "or one of the other paper-shaped fields (64^3 sine modes, the 1800x3600 climate-like and "
                        "the 100x500x500 hurricane-like field) for a trace of their kernels alone")
    p.add_argument("--n", type=int, default=512, help="edge of the cubic lognormal field")
    p.add_argument("--eb", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=300)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-configs", action="store_true", help="skip the paper-shaped fields (64^3, 1800x3600, "
                                                               "100x500x500)")
    p.add_argument("--no-layers", action="store_true", help="skip the batched and serving measurements")
    p.add_argument("--no-ablation", action="store_true", help="skip the per-kernel ablation")
    p.add_argument("--no-quality", action="store_true",
                   help="skip the rate-distortion sweep and the overall-throughput measurement")
    p.add_argument("--batch-fields", type=int, default=256)
    p.add_argument("--serve-requests", type=int, default=2000, help="requests per offered-load level")
    p.add_argument("--serve-seconds", type=float, default=4.0, help="longest trace per offered-load level")
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


def cpu_info():
    """Host facts for the CPU baseline: logical CPUs, the ones this process
    may run on, the thread budget (OMP_NUM_THREADS when set), the model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    budget = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or usable
    return {"nproc": nproc, "usable": usable, "threads": min(budget, usable), "model": model}


def cpu_baseline(x, eb, reps=3):
    """The oracle (plain C, built with OpenMP over chunks) on the same field,
    timed on the host: one single-threaded compression and decompression,
    then the best of `reps` with every thread the host grants this process
    (the box's share, OMP_NUM_THREADS).  GB/s over the input bytes;
    `value` is the all-thread round trip (compress + decompress)."""
    from oracle import oracle as O

    info = cpu_info()
    threads = info["threads"]

    def run(th):
        t0 = time.perf_counter()
        s, st = O.compress(x, eb, O.EB_REL, threads=th)
        t1 = time.perf_counter()
        _, err = O.decompress(s, x.shape, threads=th)
        t2 = time.perf_counter()
        assert st == 0 and err == 0
        return t1 - t0, t2 - t1

    tc1, td1 = run(1)
    best = min((run(threads) for _ in range(reps)), key=lambda t: t[0] + t[1])
    gb = x.nbytes / 1e9
    return {
        "value": round(gb / (best[0] + best[1]), 4),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "the whole %dx%dx%d field at REL %g: compress + decompress once with 1 thread, then best of %d "
                  "with %d OpenMP threads over chunks" % (x.shape[0], x.shape[1], x.shape[2], eb, reps, threads),
        "compress_GBps": {"threads_1": round(gb / tc1, 4), "threads_%d" % threads: round(gb / best[0], 4)},
        "decompress_GBps": {"threads_1": round(gb / td1, 4), "threads_%d" % threads: round(gb / best[1], 4)},
        "seconds": {"compress_1": round(tc1, 3), "decompress_1": round(td1, 3),
                    "compress_all": round(best[0], 3), "decompress_all": round(best[1], 3)},
        "host": info,
    }


def event_ms(fn, stream, reps):
    """Median over `reps` of the device time of fn() on `stream` (ms)."""
    import numpy as np
    import torch

    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def bench_batched(n_fields, reps=5):
    """The batch layer on 256 mixed-rank fields (16 KiB - 64 MiB, log-uniform,
    sine workload, REL eb drawn from {1e-2, 1e-3, 1e-4}): one plan run replayed
    from a graph against the same fields as plain per-field calls on one stream.
    GB/s over input bytes."""
    import torch

    import paper_2304_12557_amd as fz
    import synth

    dev = torch.device("cuda:0")
    shapes = synth.batch_shapes(n_fields=n_fields, seed=3000)
    xs = [synth.sine_field_device(sh, 3000 + i, dev) for i, sh in enumerate(shapes)]
    ebs = [synth.rel_eb_choice(3000 + i) for i in range(len(shapes))]
    nbytes = sum(4 * x.numel() for x in xs)
    st = torch.cuda.current_stream()
    plain_out = [torch.empty(fz.compress_bound(x.shape), dtype=torch.uint8, device=dev) for x in xs]
    batch_out = [torch.empty_like(o) for o in plain_out]

    def plain_c():
        for x, eb, o in zip(xs, ebs, plain_out):
            fz.compress(x, eb, "rel", out=o)

    plain_c()
    t_plain_c = event_ms(plain_c, st, reps)
    plan = fz.Batch.compress([(x, eb, "rel", o) for x, eb, o in zip(xs, ebs, batch_out)])
    plan.tune()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.run(stream=side)
    g.replay()
    torch.cuda.synchronize()
    t_batch_c = event_ms(g.replay, st, reps)
    same = all(fz.stream_size(a) == fz.stream_size(b) for a, b in zip(plain_out, batch_out))
    same = same and all(torch.equal(plain_out[i][:fz.stream_size(plain_out[i])], batch_out[i][:fz.stream_size(batch_out[i])])
                        for i in range(0, len(xs), 17))
    s_bytes = sum(fz.stream_size(o) for o in plain_out)

    ys_p = [torch.empty_like(x) for x in xs]
    ys_b = [torch.empty_like(x) for x in xs]

    def plain_d():
        for o, x, y in zip(plain_out, xs, ys_p):
            fz.decompress(o, x.shape, out=y)

    plain_d()
    t_plain_d = event_ms(plain_d, st, reps)
    dplan = fz.Batch.decompress([(o, x.shape, y, None) for o, x, y in zip(batch_out, xs, ys_b)])
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=side):
        dplan.run(stream=side)
    g2.replay()
    torch.cuda.synchronize()
    t_batch_d = event_ms(g2.replay, st, reps)
    same = same and all(torch.equal(ys_p[i].view(torch.int32), ys_b[i].view(torch.int32)) for i in range(0, len(xs), 17))
    del g, g2
    plan.close()
    dplan.close()
    gb = nbytes / 1e9
    return {
        "workload": "%d mixed-rank fields, 16 KiB-64 MiB log-uniform, sine workload, REL eb in {1e-2,1e-3,1e-4}"
                    % len(xs),
        "input_bytes": nbytes, "ratio": round(nbytes / s_bytes, 3), "identical_to_plain": bool(same),
        "compress": {"batched_GBps": round(gb / (t_batch_c * 1e-3), 1), "plain_GBps": round(gb / (t_plain_c * 1e-3), 1),
                     "batched_ms": round(t_batch_c, 3), "plain_ms": round(t_plain_c, 3)},
        "decompress": {"batched_GBps": round(gb / (t_batch_d * 1e-3), 1), "plain_GBps": round(gb / (t_plain_d * 1e-3), 1),
                       "batched_ms": round(t_batch_d, 3), "plain_ms": round(t_plain_d, 3)},
        "tuning_note": "launch shapes from fz_batch_tune; plan run replayed from a graph",
    }


def bench_serving(n_requests, max_seconds, n_pool=48, seed=4000):
    """The request server on a Poisson stream of requests (70 % compress, 30 %
    decompress) over a pool of sine-workload fields with sizes log-uniform in
    64 KiB - 256 MiB, at 25/50/90 % of the batched capacity measured on that
    pool, with a 64 GiB admission budget; against plain per-request launches on
    one stream fed by the same arrival trace.  Latency = arrival to completion
    seen by the host."""
    import ctypes
    import threading

    import numpy as np
    import torch

    import paper_2304_12557_amd as fz
    import synth

    dev = torch.device("cuda:0")
    shapes = synth.batch_shapes(n_fields=n_pool, seed=seed, lo=64 << 10, hi=256 << 20)
    xs = [synth.sine_field_device(sh, seed + i, dev) for i, sh in enumerate(shapes)]
    ebs = [synth.rel_eb_choice(seed + i) for i in range(len(xs))]
    streams = [fz.compress(x, eb, "rel") for x, eb in zip(xs, ebs)]
    torch.cuda.synchronize()
    # capacity: the whole pool as one batch (compress), bytes per second
    outs = [torch.empty_like(s) for s in streams]
    plan = fz.Batch.compress([(x, eb, "rel", o) for x, eb, o in zip(xs, ebs, outs)])
    st = torch.cuda.current_stream()
    plan.run()
    t_cap = event_ms(plan.run, st, 3)
    plan.close()
    del outs
    pool_bytes = sum(4 * x.numel() for x in xs)
    capacity = pool_bytes / (t_cap * 1e-3)
    mean_req = pool_bytes / len(xs)

    def trace(load, rs):
        rate = load * capacity / mean_req  # requests per second
        t, out = 0.0, []
        while len(out) < n_requests and t < max_seconds:
            t += rs.exponential(1.0 / rate)
            out.append((t, int(rs.integers(0, len(xs))), bool(rs.random() < 0.7)))
        return out

    def pctl(v, p):
        v = sorted(v)
        return v[min(len(v) - 1, max(0, int(np.ceil(p * len(v))) - 1))]

    L = fz.lib()
    bounds = [fz.compress_bound(x.shape) for x in xs]

    def prebuilt(tr):
        """Request structs and output buffers of a trace, made before timing."""
        reqs, keep = [], []
        for at, i, comp in tr:
            dims = fz.dims_of(xs[i].shape)
            if comp:
                o = torch.empty(bounds[i], dtype=torch.uint8, device=dev)
                r = fz.FzRequest(kind=fz.FZ_REQ_COMPRESS, eb_mode=fz.FZ_EB_REL, eb=float(ebs[i]), dims=dims,
                                 d_in=xs[i].data_ptr(), d_out=o.data_ptr(), d_err=None, hbm_bytes=0)
            else:
                o = torch.empty_like(xs[i])
                r = fz.FzRequest(kind=fz.FZ_REQ_DECOMPRESS, eb_mode=0, eb=0.0, dims=dims,
                                 d_in=streams[i].data_ptr(), d_out=o.data_ptr(), d_err=None, hbm_bytes=0,
                                 stream_bytes=streams[i].numel())
            reqs.append(r)
            keep.append(o)
        torch.cuda.synchronize()
        return reqs, keep

    def spin_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            if d > 2e-3:
                time.sleep(d - 1e-3)

    def run_server(tr):
        reqs, keep = prebuilt(tr)
        srv = fz.Server(hbm_budget=64 << 30, slots=4, max_batch=64)
        h = srv._h
        tk = ctypes.c_uint64()
        tickets = []
        t0 = time.perf_counter()
        for (at, _, _), r in zip(tr, reqs):
            spin_until(t0 + at)
            rc = L.fz_server_submit(h, ctypes.byref(r), ctypes.byref(tk))
            assert rc == 0
            tickets.append(tk.value)
        stt = ctypes.c_int()
        for t in tickets:
            L.fz_server_wait(h, t, ctypes.byref(stt))
            assert stt.value == 0
        s = srv.stats()
        srv.close()
        del keep
        return {"p50_ms": round(s["p50_ms"], 3), "p99_ms": round(s["p99_ms"], 3),
                "GBps": round(s["input_bytes"] / 1e9 / max(s["wall_s"], 1e-9), 1),
                "mean_batch": round(s["mean_batch"], 2), "admission_waits": int(s["admission_waits"])}

    def run_plain(tr):
        reqs, keep = prebuilt(tr)
        lat, done_t = [], []
        pend = []
        lock = threading.Condition()
        finished = [False]

        def poller():
            while True:
                with lock:
                    while not pend and not finished[0]:
                        lock.wait()
                    if not pend and finished[0]:
                        return
                    ev, arrival = pend[0]
                while not ev.query():
                    time.sleep(2e-5)
                now = time.perf_counter()
                with lock:
                    pend.pop(0)
                    lat.append((now - arrival) * 1e3)
                    done_t.append(now)

        th = threading.Thread(target=poller)
        th.start()
        stream = torch.cuda.Stream()
        sp = ctypes.c_void_p(stream.cuda_stream)
        evs = [torch.cuda.Event() for _ in tr]
        t0 = time.perf_counter()
        for (at, _, _), r, ev in zip(tr, reqs, evs):
            spin_until(t0 + at)
            if r.kind == fz.FZ_REQ_COMPRESS:
                rc = L.fz_compress(ctypes.c_void_p(r.d_in), ctypes.byref(r.dims), r.eb, r.eb_mode,
                                   ctypes.c_void_p(r.d_out), sp)
            else:
                rc = L.fz_decompress(ctypes.c_void_p(r.d_in), r.stream_bytes, ctypes.c_void_p(r.d_out),
                                     ctypes.byref(r.dims), None, sp)
            assert rc == 0
            ev.record(stream)
            with lock:
                pend.append((ev, t0 + at))
                lock.notify()
        with lock:
            finished[0] = True
            lock.notify()
        th.join()
        torch.cuda.synchronize()
        del keep
        nbytes = sum(4 * xs[i].numel() for _, i, _ in tr)
        wall = max(done_t) - (t0 + tr[0][0])
        return {"p50_ms": round(pctl(lat, 0.50), 3), "p99_ms": round(pctl(lat, 0.99), 3),
                "GBps": round(nbytes / 1e9 / max(wall, 1e-9), 1)}

    levels = []
    for k, load in enumerate((0.25, 0.5, 0.9)):
        tr = trace(load, np.random.default_rng(seed + 100 + k))
        levels.append({"offered_load": load, "requests": len(tr), "served": run_server(tr), "plain": run_plain(tr)})
    return {
        "workload": "Poisson stream, 70/30 compress/decompress, %d sine fields 64 KiB-256 MiB log-uniform, "
                    "64 GiB admission budget, 4 slots" % len(xs),
        "batched_capacity_GBps": round(capacity / 1e9, 1), "levels": levels,
    }

# the paper's five value-range-relative bounds (Sec. 4.1) and its host-link
# figures for the overall throughput (Sec. 4.6: PCIe 4.0 x16, and the per-GPU
# share when 4 GPUs move data at once)
REL_EBS = (1e-2, 5e-3, 1e-3, 5e-4, 1e-4)
PAPER_LINKS_GBPS = (32.0, 11.4)
PW_EPS = (1e-2, 1e-3, 1e-4)  # point-wise relative bounds of the extra mode


def rate_distortion(xt, shape):
    """Ratio, bitrate (32 / ratio) and distortion (the library's quality
    pass) of the field at each of the paper's relative bounds."""
    import torch

    import paper_2304_12557_amd as fz

    buf = torch.empty(fz.compress_bound(shape), dtype=torch.uint8, device=xt.device)
    y = torch.empty_like(xt)
    rows = []
    for eb in REL_EBS:
        fz.compress(xt, eb, "rel", out=buf)
        fz.decompress(buf, shape, out=y)
        info = fz.stream_info(buf)
        assert info["status"] == 0
        q = fz.quality(xt, y)
        ratio = 4 * xt.numel() / int(info["total_bytes"])
        eb_abs = eb * (float(info["vmax"]) - float(info["vmin"]))
        rows.append({"eb": eb, "ratio": round(ratio, 3), "bitrate": round(32.0 / ratio, 4),
                     "psnr_db": round(q["psnr"], 3), "max_abs_err": q["max_abs_err"],
                     "max_err_over_eb": round(q["max_abs_err"] / eb_abs, 6)})
    return rows


def hbm_reference(xt, y, stream, reps):
    """What plain streaming kernels reach on the same buffers (HIP events):
    a fill of the output (writes only, the decompressor's dominant traffic)
    and an elementwise copy (reads and writes).  Context for the roofline
    fractions, which are taken against the 8 TB/s peak."""
    import numpy as np
    import torch

    def timed(fn):
        fn()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
        for k in range(reps):
            ev[k][0].record(stream)
            fn()
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))

    nbytes = 4 * xt.numel()
    t_fill = timed(lambda: y.fill_(1.0))
    t_copy = timed(lambda: y.copy_(xt))
    return {"fill_GBps": round(nbytes / 1e9 / (t_fill * 1e-3), 1),
            "copy_GBps": round(2 * nbytes / 1e9 / (t_copy * 1e-3), 1),
            "note": "torch fill_ (4 B written per value) and copy_ (4 B read + 4 B written) of the benchmark field"}


def pointwise_relative(xt, shape, stream, reps):
    """The point-wise relative mode on the same field: compress and
    decompress time (HIP events), ratio, and the largest |x' - x| /
    max(|x|, 2^-126) seen (the mode's bound is eps)."""
    import numpy as np
    import torch

    import paper_2304_12557_amd as fz

    buf = torch.empty(fz.compress_bound(shape), dtype=torch.uint8, device=xt.device)
    y = torch.empty_like(xt)
    in_bytes = 4 * xt.numel()
    rows = []
    for eps in PW_EPS:
        fz.compress(xt, eps, "pwrel", out=buf)
        fz.decompress(buf, shape, out=y)
        torch.cuda.synchronize()
        info = fz.stream_info(buf)
        if info["status"]:
            rows.append({"eps": eps, "status": int(info["status"])})
            continue
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for k in range(reps):
            ev[k][0].record(stream)
            fz.compress(xt, eps, "pwrel", out=buf)
            ev[k][1].record(stream)
            fz.decompress(buf, shape, out=y)
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        tc = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        td = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        xd = xt.double()
        rel = ((y.double() - xd).abs() / xd.abs().clamp_min(2.0 ** -126)).max().item()
        del xd
        rows.append({"eps": eps, "ratio": round(in_bytes / int(info["total_bytes"]), 3),
                     "compress_GBps": round(in_bytes / 1e9 / (tc * 1e-3), 2),
                     "decompress_GBps": round(in_bytes / 1e9 / (td * 1e-3), 2),
                     "max_pointwise_rel_err": rel, "step": int(info["ebx2"])})
    return rows


def fp64_input(xt, shape, eb, stream, reps):
    """fp64 input: the same field widened to double, REL bound eb.  Compress
    and decompress time (HIP events) over the 8-byte input values, ratio,
    and the largest error over the absolute bound."""
    import numpy as np
    import torch

    import paper_2304_12557_amd as fz

    x64 = xt.double()
    buf = torch.empty(fz.compress_bound(shape, f64=True), dtype=torch.uint8, device=xt.device)
    y = torch.empty_like(x64)
    fz.compress(x64, eb, "rel", out=buf)
    fz.decompress(buf, shape, out=y)
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    if info["status"]:
        return {"eb": eb, "status": int(info["status"])}
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for k in range(reps):
        ev[k][0].record(stream)
        fz.compress(x64, eb, "rel", out=buf)
        ev[k][1].record(stream)
        fz.decompress(buf, shape, out=y)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    tc = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    td = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    in_bytes = 8 * xt.numel()
    err = (y - x64).abs().max().item()
    out = {"eb": eb, "ratio": round(in_bytes / int(info["total_bytes"]), 3),
           "compress_GBps": round(in_bytes / 1e9 / (tc * 1e-3), 2),
           "decompress_GBps": round(in_bytes / 1e9 / (td * 1e-3), 2),
           "max_err_over_eb": round(err / (0.5 * info["ebx2_f64"]), 6)}
    del x64, y, buf
    torch.cuda.empty_cache()
    return out


def global_predictor(fields, stream, reps):
    """The field-global Lorenzo predictor against the chunk-local one: ratio
    and compress / decompress rates (HIP events) per (name, tensor, REL eb)."""
    import numpy as np
    import torch

    import paper_2304_12557_amd as fz

    rows = []
    for name, xt, eb in fields:
        shape = tuple(xt.shape)
        in_bytes = 4 * xt.numel()
        row = {"field": name, "eb": eb}
        for key, glob in (("chunk_local", False), ("field_global", True)):
            buf = torch.empty(fz.compress_bound(shape, global_lorenzo=glob), dtype=torch.uint8, device=xt.device)
            y = torch.empty_like(xt)
            work = None
            if glob:
                nwork = int(fz.lib().fz_decompress_global_work_bytes(ctypes.byref(fz.dims_of(shape))))
                work = torch.empty(nwork, dtype=torch.uint8, device=xt.device)
            fz.compress(xt, eb, "rel", out=buf, global_lorenzo=glob)
            fz.decompress(buf, shape, out=y, global_lorenzo=glob, work=work)
            torch.cuda.synchronize()
            info = fz.stream_info(buf)
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
            for k in range(reps):
                ev[k][0].record(stream)
                fz.compress(xt, eb, "rel", out=buf, global_lorenzo=glob)
                ev[k][1].record(stream)
                fz.decompress(buf, shape, out=y, global_lorenzo=glob, work=work)
                ev[k][2].record(stream)
            torch.cuda.synchronize()
            tc = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
            td = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
            row[key] = {"ratio": round(in_bytes / int(info["total_bytes"]), 3),
                        "compress_GBps": round(in_bytes / 1e9 / (tc * 1e-3), 2),
                        "decompress_GBps": round(in_bytes / 1e9 / (td * 1e-3), 2)}
            del buf, y, work
        rows.append(row)
    torch.cuda.empty_cache()
    return rows


def overall_throughput(xt, shape, eb, s_bytes, t_compr_gbps, steps):
    """Overall data-transfer throughput (Sec. 4.6): compress on the device,
    then move the stream to pinned host memory.  Reports the measured
    device-to-host bandwidth, the paper's model ((BW * CR)^-1 + T^-1)^-1 at
    that bandwidth and at the paper's link figures, and the same pipeline
    timed directly (compress, then copy, back to back on one stream)."""
    import torch

    import paper_2304_12557_amd as fz

    in_bytes = 4 * xt.numel()
    ratio = in_bytes / s_bytes
    host = torch.empty(s_bytes, dtype=torch.uint8, pin_memory=True)
    buf = torch.empty(fz.compress_bound(shape), dtype=torch.uint8, device=xt.device)
    fz.compress(xt, eb, "rel", out=buf)
    src = buf[:s_bytes]
    for _ in range(2):
        host.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        host.copy_(src, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    bw = s_bytes * steps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    e0.record()
    for _ in range(steps):
        fz.compress(xt, eb, "rel", out=buf)
        host.copy_(src, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    measured = in_bytes * steps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    def model(link):
        return 1.0 / (1.0 / (link * ratio) + 1.0 / t_compr_gbps)

    return {"unit": "GB/s of input", "ratio": round(ratio, 3), "compress_GBps": round(t_compr_gbps, 2),
            "d2h_GBps": round(bw, 2), "model_GBps": round(model(bw), 2), "measured_GBps": round(measured, 2),
            "paper_links": [{"link_GBps": L, "model_GBps": round(model(L), 2)} for L in PAPER_LINKS_GBPS]}


def bench_ablation(xt, inv, t_fused_ms, reps=10):
    """The paper's per-kernel ablation (Sec. 4.5) on this field: each stage
    of the unfused pipeline timed with HIP events over `reps` launches, for
    both dual-quantization versions, both bitshuffle-mark variants and the
    encoder on either version's tiles."""
    import torch

    import paper_2304_12557_amd as fz

    ab = fz.Ablation(xt)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps  # us

    r = {}
    for v in (1, 2):
        r["pred_quant_v%d_us" % v] = timed(lambda: ab.pred_quant(v, inv))
        ab.bitshuffle_mark()
        r["encode_v%d_us" % v] = timed(ab.encode)
        r["nonzero_blocks_v%d" % v] = round(float(ab.offsets[-1].item()) / (ab.steps * 256), 4)
    # bitshuffle-mark on the v2 codes (the pipeline's state after the loop)
    ab.pred_quant(2, inv)
    r["bitshuffle_us"] = timed(ab.bitshuffle)
    r["mark_us"] = timed(ab.mark)
    r["bitshuffle_mark_v1_us"] = r["bitshuffle_us"] + r["mark_us"]
    r["bitshuffle_mark_v2_us"] = timed(ab.bitshuffle_mark)
    # the same two variants with the transpose done by wave votes (Sec. 3.3)
    r["bitshuffle_ballot_us"] = timed(lambda: ab.bitshuffle(ballot=True))
    r["bitshuffle_mark_v1_ballot_us"] = r["bitshuffle_ballot_us"] + r["mark_us"]
    r["bitshuffle_mark_v2_ballot_us"] = timed(lambda: ab.bitshuffle_mark(ballot=True))
    out = {k: (round(v, 1) if k.endswith("_us") else v) for k, v in r.items()}
    out["speedup_pred_quant"] = round(r["pred_quant_v1_us"] / r["pred_quant_v2_us"], 3)
    out["speedup_bitshuffle_mark"] = round(r["bitshuffle_mark_v1_us"] / r["bitshuffle_mark_v2_us"], 3)
    out["speedup_encode"] = round(r["encode_v1_us"] / r["encode_v2_us"], 3)
    out["speedup_swar_over_ballot_shuffle"] = round(r["bitshuffle_ballot_us"] / r["bitshuffle_us"], 3)
    out["speedup_swar_over_ballot_shuffle_mark"] = round(r["bitshuffle_mark_v2_ballot_us"] / r["bitshuffle_mark_v2_us"], 3)
    out["unfused_v2_pipeline_us"] = round(r["pred_quant_v2_us"] + r["bitshuffle_mark_v2_us"] + r["encode_v2_us"], 1)
    out["fused_compress_abs_us"] = round(t_fused_ms * 1e3, 1)
    del ab
    torch.cuda.empty_cache()
    return out


class Evictor:
    """Reads a 1 GiB scratch buffer between timed calls (outside the timed
    region) so that no input or output of the previous call is left in the
    256 MB Infinity Cache or the L2s: every timed call starts from HBM.  A
    read leaves clean lines behind, so the timed kernel pays no write-back
    of the eviction traffic."""

    def __init__(self, device, nbytes=1 << 30):
        import torch

        self.buf = torch.ones(nbytes // 4, dtype=torch.float32, device=device)

    def __call__(self):
        self.buf.amax()


def round_trips(xt, shape, eb, mode, buf, y, stream, reps, evict):
    """`reps` x (evict, compress, evict, decompress) with one pair of HIP
    events around each call on the stream the kernels run on (the end-to-end
    times), then `reps` compressions with events also between its launches
    (fz_compress_timed: the per-kernel times; each extra event costs a few
    microseconds, so these runs are not used for the end-to-end figures).
    Means in ms of: the whole compression and decompression calls, the range
    pass (k_minmax, REL; it also writes the header image and clears the
    scratch) and the main kernel (k_compress, whose last workgroup also
    settles the status word); the decompression call is its one kernel
    (k_decompress: no error word is passed)."""
    import numpy as np
    import torch

    import paper_2304_12557_amd as fz

    E = lambda: torch.cuda.Event(enable_timing=True)
    rows, parts = [], []
    for _ in range(reps):
        ev = {k: E() for k in ("c0", "c1", "d0", "d1")}
        evict()
        ev["c0"].record(stream)
        fz.compress(xt, eb, mode, out=buf, stream=stream)
        ev["c1"].record(stream)
        evict()
        ev["d0"].record(stream)
        fz.decompress(buf, shape, out=y, stream=stream)
        ev["d1"].record(stream)
        rows.append(ev)
    for _ in range(reps):
        ev = {k: E() for k in ("range_begin", "main_begin", "main_end", "done")}
        evict()
        fz.compress(xt, eb, mode, out=buf, stream=stream, events=ev)
        parts.append(ev)
    torch.cuda.synchronize()
    t = lambda rs, a, b: float(np.mean([r[a].elapsed_time(r[b]) for r in rs]))
    return {"compress": t(rows, "c0", "c1"), "decompress": t(rows, "d0", "d1"),
            "range": t(parts, "range_begin", "main_begin"), "main": t(parts, "main_begin", "main_end")}


def config_rows(stream, reps, evict):
    """The paper-shaped fields (Table 1 shapes), each alone in HBM: the small
    3-D sine field 64^3 (REL 1e-3, latency-bound), the climate-like
    1800x3600 (REL 1e-4) and the hurricane-like 100x500x500 (REL 1e-3 and
    1e-4).  Rates over the input bytes, fraction of HBM peak, ratio, and the
    main kernels' times."""
    import torch

    import paper_2304_12557_amd as fz
    import synth

    dev = torch.device("cuda:0")
    out = []
    for name, gen, eb in (("sine3d 64x64x64", synth.sine3d, 1e-3), ("climate2d 1800x3600", synth.climate2d, 1e-4),
                          ("hurricane3d 100x500x500", synth.hurricane3d, 1e-3),
                          ("hurricane3d 100x500x500", synth.hurricane3d, 1e-4)):
        x = gen()
        xt = torch.from_numpy(x).to(dev)
        shape = x.shape
        buf = torch.empty(fz.compress_bound(shape), dtype=torch.uint8, device=dev)
        y = torch.empty_like(xt)
        round_trips(xt, shape, eb, "rel", buf, y, stream, 2, evict)  # warm-up
        t = round_trips(xt, shape, eb, "rel", buf, y, stream, reps, evict)
        info = fz.stream_info(buf)
        assert info["status"] == 0
        nb = 4 * x.size
        s_bytes = int(info["total_bytes"])
        rate = lambda ms: nb / 1e9 / (ms * 1e-3)
        out.append({"workload": name, "dims": list(shape), "eb": eb, "eb_mode": "rel",
                    "ratio": round(nb / s_bytes, 3),
                    "compress_GBps": round(rate(t["compress"]), 1), "decompress_GBps": round(rate(t["decompress"]), 1),
                    "compress_pct_hbm": round(100 * rate(t["compress"]) / HBM_PEAK_GBPS, 2),
                    "decompress_pct_hbm": round(100 * rate(t["decompress"]) / HBM_PEAK_GBPS, 2),
                    "k_compress_us": round(1e3 * t["main"], 1), "k_compress_GBps": round((nb + s_bytes) / 1e9 / (t["main"] * 1e-3), 1),
                    "k_decompress_us": round(1e3 * t["decompress"], 1),
                    "k_decompress_GBps": round((nb + s_bytes) / 1e9 / (t["decompress"] * 1e-3), 1)})
        del xt, buf, y
    torch.cuda.empty_cache()
    return out


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
    if a.workload == "lognormal3d":
        x = synth.lognormal3d(seed=a.seed, n=a.n)
        wname = "lognormal3d %d^3 fp32 (cosmology-like)" % a.n
    else:
        x = getattr(synth, a.workload)()
        wname = {"sine3d": "sine3d 64x64x64 fp32 (8 sine modes + noise)",
                 "climate2d": "climate2d 1800x3600 fp32 (16 modes, 20 % exact zeros)",
                 "hurricane3d": "hurricane3d 100x500x500 fp32 (12 modes + vortex)"}[a.workload]
    shape = x.shape
    N = x.size
    in_bytes = 4 * N
    xt = torch.from_numpy(x).to(dev)
    buf = torch.empty(fz.compress_bound(shape), dtype=torch.uint8, device=dev)
    y = torch.empty(shape, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    evict = Evictor(dev)

    for _ in range(a.warmup):
        fz.compress(xt, a.eb, "rel", out=buf)
        fz.decompress(buf, shape, out=y)
    torch.cuda.synchronize()
    if a.calib_copy:
        ycopy = torch.empty_like(xt)
        torch.neg(xt, out=ycopy)  # an elementwise kernel of its own name: 4N bytes in, 4N out
        torch.cuda.synchronize()
        del ycopy
    info = fz.stream_info(buf)
    assert info["status"] == 0
    s_bytes = int(info["total_bytes"])

    # the timed steps: REL compression then decompression of the field, each
    # preceded (outside its events) by a 1 GiB read that evicts the caches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rel = round_trips(xt, shape, a.eb, "rel", buf, y, stream, a.steps, evict)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    tc, td = rel["compress"], rel["decompress"]
    # ABS mode with the absolute bound the relative one produced (no range pass)
    eb_abs = a.eb * (float(info["vmax"]) - float(info["vmin"]))
    ab = round_trips(xt, shape, eb_abs, "abs", buf, y, stream, a.steps, evict)
    assert fz.stream_info(buf)["total_bytes"] == s_bytes
    t_ev = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        evict()
        e1.record(stream)
        torch.cuda.synchronize()
        t_ev.append(e0.elapsed_time(e1))

    # roofline: every kernel of the step with its algorithmic bytes and its
    # mean launch time from the events that bracket it; the dominant one (the
    # longest) is the headline entry
    kernels = [
        ("k_compress", in_bytes + s_bytes, (rel["main"] + ab["main"]) / 2,
         "4N read + S_c written (placed payload)"),
        ("k_decompress", in_bytes + s_bytes, (rel["decompress"] + ab["decompress"]) / 2, "S_c read + 4N written"),
        ("k_minmax", in_bytes, rel["range"], "4N read (REL range pass)"),
    ]
    krows = []
    for name, alg, t_ms, what in kernels:
        ach = alg / (t_ms * 1e-3) / 1e9
        krows.append({"kernel": name, "algorithmic_bytes": int(alg), "bytes": what, "avg_launch_ms": round(t_ms, 4),
                      "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBPS, 4)})
    dom = max(krows, key=lambda r: r["avg_launch_ms"])
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
        "config": {"workload": "%s, REL eb %g, compress + decompress" % (wname, a.eb), "dims": list(shape),
                   "eb": a.eb, "eb_mode": "rel"},
        "timing_note": "each compression and decompression is preceded, outside its events, by a 1 GiB read that "
                       "evicts the caches (%.3f ms, inside ms_per_step twice per step)" % float(np.mean(t_ev)),
        "compress_GBps": round(in_bytes / 1e9 / (tc * 1e-3), 2),
        "compress_abs_GBps": round(in_bytes / 1e9 / (ab["compress"] * 1e-3), 2),
        "decompress_GBps": round(in_bytes / 1e9 / (td * 1e-3), 2),
        "compress_pct_hbm": round(100 * in_bytes / 1e9 / (tc * 1e-3) / HBM_PEAK_GBPS, 2),
        "compress_abs_pct_hbm": round(100 * in_bytes / 1e9 / (ab["compress"] * 1e-3) / HBM_PEAK_GBPS, 2),
        "decompress_pct_hbm": round(100 * in_bytes / 1e9 / (td * 1e-3) / HBM_PEAK_GBPS, 2),
        "end_to_end_target": "ABS compression >= 50 %% of HBM peak over the input bytes (t <= %.0f us here)"
                             % (in_bytes / 4e12 * 1e6),
        "ratio": round(in_bytes / s_bytes, 3),
        "stream_bytes": s_bytes,
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["achieved"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": dom["frac"],
                     "traffic": measured_traffic(dom["kernel"], shape, a.eb) if dom["kernel"] in KERNEL_SOURCES else None,
                     "algorithmic_bytes": dom["algorithmic_bytes"], "avg_launch_ms": dom["avg_launch_ms"]},
        "kernels": krows,
    }
    out["hbm_reference"] = hbm_reference(xt, y, stream, a.steps)
    if not a.no_configs:
        out["configs"] = config_rows(stream, a.steps, evict)
    if not a.no_quality:
        out["rate_distortion"] = rate_distortion(xt, shape)
        out["overall_throughput"] = overall_throughput(xt, shape, a.eb, s_bytes, in_bytes / 1e9 / (tc * 1e-3),
                                                       a.steps)
        out["pointwise_relative"] = pointwise_relative(xt, shape, stream, a.steps)
        out["fp64_input"] = fp64_input(xt, shape, a.eb, stream, a.steps)
        hur = torch.from_numpy(synth.hurricane3d()).to(dev)
        out["global_predictor"] = global_predictor([(wname.split(" fp32")[0], xt, a.eb),
                                                    ("hurricane3d 100x500x500", hur, 1e-3)], stream, a.steps)
        del hur
    if not a.no_ablation:
        out["ablation"] = bench_ablation(xt, float(info["inv"]), ab["compress"])
    if not a.no_layers:
        del buf, y, evict
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(a.batch_fields)
        torch.cuda.empty_cache()
        out["serving"] = bench_serving(a.serve_requests, a.serve_seconds)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, a.eb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
