"""GPU parity of the field-global Lorenzo predictor (fz_compress_global /
fz_decompress_global) through the C ABI.

The bar is that of the other parity tests: the oracle's status, and when it
is 0 the same stream bytes and the same reconstruction bits.  Cases: the
three ranks with whole and ragged chunk grids (several chunks along every
axis, so that every face carries), contiguous extents that are not
multiples of 4, the three bound modes, statuses, streams of the other
predictor, and the whole hurricane-like field.
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
MODES = {O.EB_ABS: "abs", O.EB_REL: "rel", O.EB_PWREL: "pwrel"}


def gpu_run(x, eb, mode):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    buf = fz.compress(xt, eb, MODES[mode], global_lorenzo=True)
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    if info["status"]:
        return info["status"], None, None, None
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, x.shape, err=err, global_lorenzo=True)
    torch.cuda.synchronize()
    n = int(info["total_bytes"])
    return 0, buf[:n].cpu().numpy(), y.cpu().numpy(), int(err.item())


def check(x, eb, mode, threads=1):
    print("global case", x.shape, eb, mode, flush=True)
    ref, st = O.compress(x, eb, mode, threads=threads, global_lorenzo=True)
    gst, s, y, err = gpu_run(x, eb, mode)
    assert gst == st == 0, (gst, st)
    assert s.size == ref.size, (s.size, ref.size)
    if not np.array_equal(s, ref):
        diff = np.nonzero(s != ref)[0]
        raise AssertionError("stream differs at %d bytes, first at %d of %d" % (diff.size, diff[0], s.size))
    assert err == 0
    yo, erro = O.decompress(ref, x.shape)
    assert erro == 0
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))
    return s


@pytest.mark.parametrize("shape,eb,mode", [
    ((40, 70, 130), 1e-3, O.EB_REL),   # 3 x 3 x 3 chunks, ragged in every dimension
    ((16, 32, 64), 1e-3, O.EB_ABS),    # one chunk: the chunk-local stream but for byte 15
    ((33, 65, 131), 1e-2, O.EB_REL),   # contiguous extent odd (scalar loads)
    ((70, 2100), 1e-3, O.EB_ABS),      # 2-D, 3 x 3 chunks
    ((45, 1027), 1e-4, O.EB_REL),      # 2-D, contiguous extent not a multiple of 4
    ((100000,), 1e-4, O.EB_REL),       # 1-D, 4 chunks
    ((65537,), 1e-3, O.EB_ABS),        # 1-D, two chunks and one value
    ((1,), 1e-3, O.EB_REL), ((3, 1, 5), 1e-3, O.EB_ABS),
])
def test_parity(shape, eb, mode):
    check(synth.sine_field(shape, seed=sum(shape)), eb, mode)


def test_pointwise_relative_mode():
    check(synth.wide_field((40, 70, 130), seed=12), 1e-2, O.EB_PWREL)


def test_statuses():
    x = synth.sine_field((40, 70, 130), seed=13)
    for v in (np.nan, np.inf):
        bad = x.copy()
        bad[20, 35, 64] = v  # on chunk faces: the neighbours' predictions read it too
        for mode in (O.EB_ABS, O.EB_REL):
            _, st = O.compress(bad, 1e-3, mode, global_lorenzo=True)
            assert gpu_run(bad, 1e-3, mode)[0] == st == O.ERR_NONFINITE
    big = x * np.float32(1e30)
    _, st = O.compress(big, 1e-10, O.EB_ABS, global_lorenzo=True)
    assert gpu_run(big, 1e-10, O.EB_ABS)[0] == st == O.ERR_EB_RANGE
    w = (np.random.default_rng(3).standard_normal((40, 70, 130)) * 1e6).astype(np.float32)
    _, st = O.compress(w, 0.5, O.EB_ABS, global_lorenzo=True)
    assert gpu_run(w, 0.5, O.EB_ABS)[0] == st == O.ERR_OUTLIER_CAP


def test_predictors_do_not_mix():
    x = synth.sine_field((40, 70, 130), seed=14)
    xt = torch.from_numpy(x).cuda()
    sl = fz.compress(xt, 1e-3, "rel")
    sg = fz.compress(xt, 1e-3, "rel", global_lorenzo=True)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    fz.decompress(sg, x.shape, err=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 6
    fz.decompress(sl, x.shape, err=err, global_lorenzo=True)
    torch.cuda.synchronize()
    assert int(err.item()) == 6
    assert fz.stream_info(sg)["predictor"] == 1 and fz.stream_info(sl)["predictor"] == 0
    # the same reconstruction from either stream
    ya = fz.decompress(sl, x.shape)
    yb = fz.decompress(sg, x.shape, global_lorenzo=True)
    torch.cuda.synchronize()
    assert torch.equal(ya.view(torch.int32), yb.view(torch.int32))


def test_full_size_hurricane():
    """100 x 500 x 500, REL 1e-3: whole stream and reconstruction."""
    x = synth.hurricane3d()
    s = check(x, 1e-3, O.EB_REL, threads=THREADS)
    sl, _ = O.compress(x, 1e-3, O.EB_REL, threads=THREADS)
    print("ratio chunk-local %.3f, field-global %.3f" % (x.nbytes / sl.size, x.nbytes / s.size), flush=True)
