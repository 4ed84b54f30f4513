"""A seeded sweep of the GPU path against the oracle through the C ABI.

Each case draws a rank, extents (often a chunk box plus or minus one, and
contiguous extents that are not multiples of 4), a value recipe, an error-bound
mode and a bound, all from a fixed seed.  The recipes include smooth modes,
heavy-tailed lognormal values, white noise (escapes, and at small bounds the
escape cap), blocks of exact zeros, signed zeros, constant patches and fp32
denormals.  The bar is that of the parity tests: the same status as the
oracle, and when it is 0, the same stream bytes and the same reconstruction
bits.
"""
import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu

from synth import draw_field, draw_shape

def gpu_run(x, eb, mode):
    xt = torch.from_numpy(x).cuda()
    buf = fz.compress(xt, eb, "rel" if mode == O.EB_REL else "abs")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    if info["status"]:
        return info["status"], None, None, None
    y = fz.decompress(buf, x.shape, err=err)
    torch.cuda.synchronize()
    n = int(info["total_bytes"])
    return 0, buf[:n].cpu().numpy(), y.cpu().numpy(), int(err.item())


@pytest.mark.parametrize("case", range(40))
def test_sweep(case):
    rng = np.random.default_rng(7000 + case)
    rank = int(rng.integers(1, 4))
    shape = draw_shape(rng, rank)
    kind, x = draw_field(rng, shape, 7000 + case)
    mode = O.EB_REL if rng.random() < 0.7 else O.EB_ABS
    eb = float(10 ** rng.uniform(-5, -1))
    if mode == O.EB_ABS:
        span = float(np.max(x) - np.min(x))
        eb = eb * (span if span > 0 else 1.0)
        if eb < 1e-37:
            eb = 1e-37
    print("sweep case", case, shape, kind, "rel" if mode == O.EB_REL else "abs", eb, flush=True)
    ref, st = O.compress(x, eb, mode)
    gst, s, y, err = gpu_run(x, eb, mode)
    assert gst == st, (gst, st)
    if st:
        return
    assert s.size == ref.size and np.array_equal(s, ref)
    assert err == 0
    yo, erro = O.decompress(ref, shape)
    assert erro == 0
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))


def test_sweep_escape_cap_and_denormal_range():
    """Noise far above the bound exceeds the escape cap; a field of denormals
    alone in REL mode gives a bound below the smallest normal fp32 (EB_RANGE);
    in ABS mode it compresses."""
    rng = np.random.default_rng(7100)
    noise = (rng.standard_normal((16, 32, 64)) * 1e6).astype(np.float32)
    den = (synth.sine_field((20, 33, 70), seed=7101) * np.float32(1e-39)).astype(np.float32)
    for x, eb, mode, want in ((noise, 0.5, O.EB_ABS, O.ERR_OUTLIER_CAP), (den, 1e-3, O.EB_REL, O.ERR_EB_RANGE),
                              (den, 1e-37, O.EB_ABS, 0)):
        ref, st = O.compress(x, eb, mode)
        gst, s, y, err = gpu_run(x, eb, mode)
        assert st == gst == want
        if st == 0:
            assert np.array_equal(s, ref)
            yo, _ = O.decompress(ref, x.shape)
            assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))
