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
    p.add_argument("--n", type=int, default=512, help="edge of the cubic lognormal field")
    p.add_argument("--eb", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=300)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum CPU time of the oracle baseline")
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
                                 d_in=streams[i].data_ptr(), d_out=o.data_ptr(), d_err=None, hbm_bytes=0)
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
                rc = L.fz_decompress(ctypes.c_void_p(r.d_in), ctypes.c_void_p(r.d_out), ctypes.byref(r.dims), None, sp)
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
    out = {k: (round(v, 1) if k.endswith("_us") else v) for k, v in r.items()}
    out["speedup_pred_quant"] = round(r["pred_quant_v1_us"] / r["pred_quant_v2_us"], 3)
    out["speedup_bitshuffle_mark"] = round(r["bitshuffle_mark_v1_us"] / r["bitshuffle_mark_v2_us"], 3)
    out["speedup_encode"] = round(r["encode_v1_us"] / r["encode_v2_us"], 3)
    out["unfused_v2_pipeline_us"] = round(r["pred_quant_v2_us"] + r["bitshuffle_mark_v2_us"] + r["encode_v2_us"], 1)
    out["fused_compress_abs_us"] = round(t_fused_ms * 1e3, 1)
    del ab
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
    out["hbm_reference"] = hbm_reference(xt, y, stream, a.steps)
    if not a.no_quality:
        out["rate_distortion"] = rate_distortion(xt, shape)
        out["overall_throughput"] = overall_throughput(xt, shape, a.eb, s_bytes, in_bytes / 1e9 / (tc * 1e-3),
                                                       a.steps)
        out["pointwise_relative"] = pointwise_relative(xt, shape, stream, a.steps)
        out["fp64_input"] = fp64_input(xt, shape, a.eb, stream, a.steps)
        hur = torch.from_numpy(synth.hurricane3d()).to(dev)
        out["global_predictor"] = global_predictor([("lognormal3d %d^3" % a.n, xt, a.eb),
                                                    ("hurricane3d 100x500x500", hur, 1e-3)], stream, a.steps)
        del hur
    if not a.no_ablation:
        out["ablation"] = bench_ablation(xt, float(info["inv"]), tca)
    if not a.no_layers:
        del buf, y
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(a.batch_fields)
        torch.cuda.empty_cache()
        out["serving"] = bench_serving(a.serve_requests, a.serve_seconds)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, a.eb, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
