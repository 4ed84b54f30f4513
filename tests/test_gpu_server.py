"""The request server on the GPU (continuous batching with HBM admission).

* Compress and decompress requests of mixed rank and size, arriving with
  random gaps, give exactly the oracle's results and the per-field call's
  (streams byte for byte, reconstructions bit for bit): each result is the
  same alone and in the mix.
* A request submitted right after its input is produced on the caller's
  stream, with no synchronization, reads the finished input (the request
  waits for the caller's stream on the device).
* With a budget smaller than the requests' total, requests wait for
  admission, the admitted bytes never exceed the budget, and the results are
  unchanged.
* Two host threads submitting at once get correct results.
"""
import threading
import time

import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu


def requests(n=24, seed=4000, host=False):
    shapes = synth.batch_shapes(n_fields=n, seed=seed, lo=64 << 10, hi=8 << 20)
    out = []
    for i, sh in enumerate(shapes):
        xh = synth.batch_field(sh, seed + i)
        x = torch.from_numpy(xh).cuda()
        out.append((x, synth.rel_eb_choice(seed + i)) + ((xh,) if host else ()))
    return out


def plain(x, eb):
    s = fz.compress(x, eb, "rel")
    y = fz.decompress(s, x.shape)
    torch.cuda.synchronize()
    n = fz.stream_size(s)
    return s[:n].clone(), y


def test_server_results_equal_plain_calls():
    reqs_h = requests(host=True)
    reqs = [(x, eb) for x, eb, _ in reqs_h]
    ref = [plain(x, eb) for x, eb in reqs]
    # the per-field results are the oracle's
    oracle = []
    for (x, eb, xh), (s, y) in zip(reqs_h, ref):
        o, st = O.compress(xh, eb, O.EB_REL)
        yo, err = O.decompress(o, xh.shape)
        assert st == 0 and err == 0
        assert np.array_equal(s.cpu().numpy(), o)
        oracle.append((o, yo))
    srv = fz.Server(hbm_budget=64 << 30, slots=4, max_batch=8)
    rng = np.random.default_rng(7)
    tickets = []
    for i, (x, eb) in enumerate(reqs):  # compress all, decompress every third stream, with gaps
        tickets.append(("c", i, srv.submit_compress(x, eb, "rel")))
        if i % 3 == 0:
            tickets.append(("d", i, srv.submit_decompress(ref[i][0], x.shape)))
        time.sleep(float(rng.exponential(2e-4)))
    for kind, i, t in tickets:
        out = srv.wait(t)
        if kind == "c":
            n = fz.stream_size(out)
            assert n == ref[i][0].numel() and torch.equal(out[:n], ref[i][0]), i
            assert np.array_equal(out[:n].cpu().numpy(), oracle[i][0]), i
        else:
            assert torch.equal(out.view(torch.int32), ref[i][1].view(torch.int32)), i
            assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle[i][1].view(np.uint32)), i
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["queued"] == 0
    assert st["batches"] >= 1 and st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_server_admission_budget():
    reqs = requests(n=12, seed=4100)
    ref = [plain(x, eb)[0] for x, eb in reqs]
    sizes = [4 * x.numel() + fz.compress_bound(x.shape) for x, _ in reqs]
    budget = max(sizes) + min(sizes)  # at most a couple of requests admitted at once
    srv = fz.Server(hbm_budget=budget, slots=4, max_batch=8)
    ts = [srv.submit_compress(x, eb, "rel") for x, eb in reqs]
    for i, t in enumerate(ts):
        out = srv.wait(t)
        n = fz.stream_size(out)
        assert torch.equal(out[:n], ref[i]), i
    st = srv.stats()
    assert st["admission_waits"] > 0
    assert st["inflight_max_bytes"] <= budget
    srv.close()


def test_server_two_submitting_threads():
    reqs = requests(n=16, seed=4200)
    ref = [plain(x, eb)[0] for x, eb in reqs]
    srv = fz.Server(hbm_budget=64 << 30, slots=2, max_batch=4)
    got = {}

    def client(idx):
        ts = [(i, srv.submit_compress(reqs[i][0], reqs[i][1], "rel")) for i in idx]
        for i, t in ts:
            got[i] = srv.wait(t)

    th = [threading.Thread(target=client, args=(list(range(k, len(reqs), 2)),)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, r in enumerate(ref):
        n = fz.stream_size(got[i])
        assert torch.equal(got[i][:n], r), i
    srv.close()


def test_server_waits_for_the_callers_stream():
    """The input is produced by kernels still queued on the current stream
    when the request is submitted (no synchronization in between); the
    result is that of the finished input."""
    x0 = torch.from_numpy(synth.sine_field((64, 96, 200), seed=4300)).cuda()
    ref, _ = plain(x0, 1e-3)
    srv = fz.Server(hbm_budget=64 << 30, slots=2, max_batch=4)
    torch.cuda.synchronize()
    for rep in range(3):
        x = torch.zeros_like(x0)
        # a long chain of small kernels on the current stream before x is final
        for _ in range(200):
            x.mul_(1.0)
        x.copy_(x0)
        t = srv.submit_compress(x, 1e-3, "rel")  # no sync: the request must wait for the copy
        out = srv.wait(t)
        n = fz.stream_size(out)
        assert n == ref.numel() and torch.equal(out[:n], ref), rep
    srv.close()
