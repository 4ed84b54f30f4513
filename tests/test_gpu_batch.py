"""The batch layer on the GPU.

* Every field of a mixed batch (ranks 1-3, aligned and unaligned rows, REL
  and ABS bounds, sizes from one chunk to several hundred) gets exactly the
  oracle's bytes and the per-field call's; the batched decompression gives
  the oracle's reconstruction and the per-field call's, bit for bit.
* The benchmark's batch (256 fields of 16 KiB - 64 MiB, 2.6 GB) against the
  oracle, field by field, in both directions.
* A field whose REL pass fails (NaN) gets the per-field status; its
  neighbours in the batch are unaffected.
* A run captured in a graph and replayed several times, with eager work in
  between, matches the eager run every time; tuning changes no byte.
"""
import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu


def mixed_batch(n=18, seed=3000, lo=16 << 10, hi=4 << 20):
    shapes = synth.batch_shapes(n_fields=n, seed=seed, lo=lo, hi=hi)
    shapes += [(37, 70, 130), (75, 2050), (100001,), (16, 32, 64)]  # unaligned rows, exact chunk
    fields, ebs, modes = [], [], []
    for i, sh in enumerate(shapes):
        x = synth.batch_field(sh, seed + i)
        rel = synth.rel_eb_choice(seed + i)
        mode = "abs" if i % 5 == 4 else "rel"
        eb = rel if mode == "rel" else rel * float(x.max() - x.min())
        fields.append(x)
        ebs.append(eb)
        modes.append(mode)
    return fields, ebs, modes


def plain_streams(xs, ebs, modes):
    out = []
    for x, eb, mode in zip(xs, ebs, modes):
        buf = fz.compress(x, eb, mode)
        torch.cuda.synchronize()
        out.append(buf[:fz.stream_size(buf)].cpu().numpy())
    return out


def batch_streams(outs):
    torch.cuda.synchronize()
    return [o[:fz.stream_size(o)].cpu().numpy() for o in outs]


@pytest.fixture(scope="module")
def batch():
    fields, ebs, modes = mixed_batch()
    xs = [torch.from_numpy(f).cuda() for f in fields]
    return fields, xs, ebs, modes


def test_batch_compress_equals_plain_calls(batch):
    fields, xs, ebs, modes = batch
    print("batch of", len(xs), "fields", flush=True)
    ref = plain_streams(xs, ebs, modes)
    b = fz.Batch.compress([(x, eb, m, None) for x, eb, m in zip(xs, ebs, modes)])
    got = batch_streams(b.run())
    for i, (r, s) in enumerate(zip(ref, got)):
        assert r.size == s.size and np.array_equal(r, s), (i, fields[i].shape)
    for i in range(len(fields)):  # and the oracle, on every field
        o, st = O.compress(fields[i], ebs[i], O.EB_REL if modes[i] == "rel" else O.EB_ABS)
        assert st == 0 and np.array_equal(o, got[i]), i
    b.close()


def test_batch_decompress_equals_plain_calls(batch):
    fields, xs, ebs, modes = batch
    bufs = [fz.compress(x, eb, m) for x, eb, m in zip(xs, ebs, modes)]
    ref = [fz.decompress(s, f.shape) for s, f in zip(bufs, fields)]
    errs = [torch.ones(1, dtype=torch.int32, device="cuda") for _ in bufs]
    b = fz.Batch.decompress([(s, f.shape, None, e) for s, f, e in zip(bufs, fields, errs)])
    ys = b.run()
    torch.cuda.synchronize()
    for i, (r, y, e) in enumerate(zip(ref, ys, errs)):
        assert int(e.item()) == 0
        assert torch.equal(r.view(torch.int32), y.view(torch.int32)), i
    # and the oracle's reconstruction of the oracle's stream, on every field
    for i, f in enumerate(fields):
        o, st = O.compress(f, ebs[i], O.EB_REL if modes[i] == "rel" else O.EB_ABS)
        yo, err = O.decompress(o, f.shape)
        assert st == 0 and err == 0
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint32), yo.view(np.uint32)), i
    b.close()


def test_batch_benchmark_scale_against_oracle():
    """The benchmark's batch: 256 fields of rank 1-3 with log-uniform sizes
    of 16 KiB - 64 MiB (2.6 GB in all), sine workload generated on the device
    and copied to the host for the oracle, REL bounds from {1e-2, 1e-3, 1e-4}.
    One batched compression and one batched decompression, every field
    against the oracle (threaded compression, single-threaded decompression)."""
    import os

    threads = min(os.cpu_count() or 1, 16)
    dev = torch.device("cuda")
    shapes = synth.batch_shapes(n_fields=256, seed=3000)
    xs = [synth.sine_field_device(sh, 3000 + i, dev) for i, sh in enumerate(shapes)]
    ebs = [synth.rel_eb_choice(3000 + i) for i in range(len(shapes))]
    print("benchmark batch: %d fields, %.2f GB" % (len(xs), sum(4 * x.numel() for x in xs) / 1e9), flush=True)
    b = fz.Batch.compress([(x, eb, "rel", None) for x, eb in zip(xs, ebs)])
    outs = b.run()
    torch.cuda.synchronize()
    streams = [o[:fz.stream_size(o)].clone() for o in outs]
    b.close()
    del outs
    errs = [torch.ones(1, dtype=torch.int32, device=dev) for _ in xs]
    d = fz.Batch.decompress([(s, x.shape, None, e) for s, x, e in zip(streams, xs, errs)])
    ys = d.run()
    torch.cuda.synchronize()
    for i, (x, eb) in enumerate(zip(xs, ebs)):
        xh = x.cpu().numpy()
        o, st = O.compress(xh, eb, O.EB_REL, threads=threads)
        assert st == 0
        s = streams[i].cpu().numpy()
        assert s.size == o.size and np.array_equal(s, o), (i, shapes[i])
        assert int(errs[i].item()) == 0, i
        yo, err = O.decompress(o, xh.shape)
        assert err == 0 and np.array_equal(ys[i].cpu().numpy().view(np.uint32), yo.view(np.uint32)), (i, shapes[i])
    d.close()


def test_batch_failing_field_is_isolated():
    a = synth.sine_field((20, 40, 70), seed=1)
    bad = a.copy()
    bad[3, 5, 7] = np.nan
    c = synth.sine_field((3000,), seed=2)
    xs = [torch.from_numpy(v).cuda() for v in (a, bad, c)]
    b = fz.Batch.compress([(x, 1e-3, "rel", None) for x in xs])
    outs = b.run()
    torch.cuda.synchronize()
    infos = [fz.stream_info(o) for o in outs]
    assert infos[0]["status"] == 0 and infos[2]["status"] == 0
    assert infos[1]["status"] == fz.STATUS_NONFINITE
    ref = plain_streams([xs[0], xs[2]], [1e-3, 1e-3], ["rel", "rel"])
    got = batch_streams([outs[0], outs[2]])
    assert all(np.array_equal(r, s) for r, s in zip(ref, got))
    b.close()


def test_batch_graph_replay_and_tuning(batch):
    fields, xs, ebs, modes = batch
    sub = list(range(0, len(xs), 2))
    jobs = [(xs[i], ebs[i], modes[i], None) for i in sub]
    b = fz.Batch.compress(jobs)
    b.tune()
    eager = batch_streams(b.run())
    ref = plain_streams([xs[i] for i in sub], [ebs[i] for i in sub], [modes[i] for i in sub])
    assert all(np.array_equal(r, s) for r, s in zip(ref, eager))
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        b.run(stream=side)
    for rep in range(3):
        for o in b.outs:
            o.fill_(0xAB)  # eager work between replays: clobber the outputs
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = batch_streams(b.outs)
        for i, (r, s) in enumerate(zip(eager, got)):
            assert np.array_equal(r, s), (rep, i)
    del g
    b.close()
