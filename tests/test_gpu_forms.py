"""GPU parity of every launch form of the decompressor against the oracle.

The library decompresses a field with one wave per chunk when it has many
chunks, and with a workgroup of 4 waves per chunk (each on one of the chunk's
layers, the carries between them exchanged in LDS) when it has at most 512.
Each rank gets fields, ragged against the chunk box, on both sides of that
line; the bar is the usual one: the whole stream byte for byte and the whole
reconstruction bit for bit.  The point-wise relative mode runs through the
same forms with its own dequantization, so it gets a case of each form too.
"""
import os

import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu

THREADS = min(os.cpu_count() or 1, 16)


def chunks(shape):
    box = {1: (32768,), 2: (32, 1024), 3: (16, 32, 64)}[len(shape)]
    n = 1
    for s, b in zip(shape, box):
        n *= -(-s // b)
    return n


def form(shape):
    return 4 if chunks(shape) <= 512 else 1


CASES = [
    ((9_830_401,), 4),          # 1-D, 301 chunks, the last one value long
    ((16_777_217,), 1),         # 1-D, 512 whole chunks and one value: 513
    ((36_000_001,), 1),         # 1-D, 1099 chunks
    ((511, 32_700), 4),         # 2-D, 16 x 32 = 512 chunks, both cut
    ((630, 30_000), 1),         # 2-D, 20 x 30 chunks, both cut
    ((100, 300, 500), 1),       # 3-D, 7 x 10 x 8 chunks, all three cut
    ((60, 300, 500), 4),        # 3-D, 4 x 10 x 8 chunks, all three cut
]


@pytest.mark.parametrize("shape,nw", CASES)
def test_forms_rel(shape, nw):
    assert form(shape) == nw, (shape, chunks(shape))
    x = synth.sine_field(shape, seed=7000 + len(shape))
    print("case", shape, "chunks", chunks(shape), "waves per chunk", nw, flush=True)
    ref, st = O.compress(x, 1e-3, O.EB_REL, threads=THREADS)
    assert st == 0
    xt = torch.from_numpy(x).cuda()
    buf = fz.compress(xt, 1e-3, "rel")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, shape, err=err)
    torch.cuda.synchronize()
    n = fz.stream_size(buf)
    s = buf[:n].cpu().numpy()
    assert int(err.item()) == 0
    assert s.size == ref.size and np.array_equal(s, ref)
    yo, e = O.decompress(ref, shape, threads=THREADS)
    assert e == 0
    assert np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32))


@pytest.mark.parametrize("shape,nw", [((40, 300, 300), 4), ((100, 300, 500), 1), ((1_100, 33_000), 1)])
def test_forms_pointwise_relative(shape, nw):
    assert form(shape) == nw
    rng = np.random.default_rng(8000 + len(shape))
    x = (np.exp(synth.sine_field(shape, seed=8100).astype(np.float64)) *
         rng.choice([-1.0, 1.0], size=1)).astype(np.float32)  # one sign: few escapes
    print("case", shape, "chunks", chunks(shape), "waves per chunk", nw, flush=True)
    ref, st = O.compress(x, 1e-3, O.EB_PWREL, threads=THREADS)
    assert st == 0
    xt = torch.from_numpy(x).cuda()
    buf = fz.compress(xt, 1e-3, "pwrel")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, shape, err=err)
    torch.cuda.synchronize()
    n = fz.stream_size(buf)
    assert int(err.item()) == 0
    assert np.array_equal(buf[:n].cpu().numpy(), ref)
    yo, e = O.decompress(ref, shape, threads=THREADS)
    assert e == 0
    assert np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32))
