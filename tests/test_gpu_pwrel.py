"""GPU parity of the point-wise relative mode (FZ_EB_PWREL) through the C ABI.

The pipeline is the same as in the other modes, on the float's bit pattern
with the step S of the relative bound (integer arithmetic only), so the bar
is the same: the oracle's status, and when it is 0 the same stream bytes and
the same reconstruction bits.  Cases: the three ranks with whole and ragged
chunk boxes, contiguous extents that are not multiples of 4 (the scalar
load path), the smallest and largest steps, the workload of positive values
over several binades at 512^3, and the statuses (non-finite input, a bound
whose step is below 2, the escape cap for white noise that changes sign).
The reconstruction is also checked against the bound itself.
"""
import os

import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu

FLT_MIN = 2.0 ** -126
THREADS = min(os.cpu_count() or 1, 16)


def gpu_run(x, eps):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    buf = fz.compress(xt, eps, "pwrel")
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    if info["status"]:
        return info["status"], None, None, None
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, x.shape, err=err)
    torch.cuda.synchronize()
    n = int(info["total_bytes"])
    return 0, buf[:n].cpu().numpy(), y.cpu().numpy(), int(err.item())


def check(x, eps, threads=1):
    print("pwrel case", x.shape, eps, flush=True)
    ref, st = O.compress(x, eps, O.EB_PWREL, threads=threads)
    gst, s, y, err = gpu_run(x, eps)
    assert gst == st == 0, (gst, st)
    assert s.size == ref.size, (s.size, ref.size)
    if not np.array_equal(s, ref):
        diff = np.nonzero(s != ref)[0]
        raise AssertionError("stream differs at %d bytes, first at %d of %d" % (diff.size, diff[0], s.size))
    assert err == 0
    yo, erro = O.decompress(ref, x.shape)
    assert erro == 0
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    assert np.all(np.abs(yd - xd) <= eps * np.maximum(np.abs(xd), FLT_MIN))
    return s


@pytest.mark.parametrize("shape,eps", [
    ((20, 40, 70), 1e-3),      # 3-D, ragged in every dimension
    ((16, 32, 64), 0.3),       # one whole chunk box
    ((33, 65, 131), 1e-2),     # box + 1, contiguous extent odd (scalar loads)
    ((45, 1030), 1e-2),        # 2-D ragged
    ((33, 1027), 1e-3),        # 2-D, contiguous extent not a multiple of 4
    ((70001,), 1e-4),          # 1-D ragged
    ((65537,), 1e-2),          # 1-D, two chunks and one value
    ((1,), 1e-3), ((3, 1, 5), 1e-3),
])
def test_parity(shape, eps):
    check(synth.wide_field(shape, seed=sum(shape)), eps)


def test_step_extremes():
    # S = 2 (eps just above 2^-23): a nearly constant field keeps the deltas small
    x = (1.0 + 1e-5 * synth.sine_field((20, 40, 70), seed=5)).astype(np.float32)
    s = check(x, 1.2e-7)
    assert fz.stream_info(torch.from_numpy(s).cuda())["ebx2"] == 2.0
    # S just below 2^24 (eps = 1e6): codes 0 / +-1 per binade-sized step
    s = check(synth.wide_field((20, 40, 70), seed=6), 1e6)
    assert fz.stream_info(torch.from_numpy(s).cuda())["ebx2"] == float(np.floor(1e6 * 2 ** 24 / (1 + 1e6)))


def test_zeros_signed_zeros_and_denormals():
    x = synth.wide_field((20, 40, 70), seed=7)
    x[:5] = 0.0
    x[5:7] = np.float32(-0.0)
    x[10, :, :8] = np.float32(1.5e-45)  # the smallest denormal
    check(x, 1e-3)


def test_statuses():
    # this field's sign regions put 287 escapes in one layer (859 in its
    # chunk, within the chunk's allowance of 1024): a valid stream
    x = synth.wide_field((20, 40, 70), seed=8)
    s = check(x, 1e-3)
    assert fz.stream_info(torch.from_numpy(s).cuda())["n_outliers"] > 1024
    # a non-finite value ends the pipeline first, so only its bit is set
    for v in (np.nan, np.inf, -np.inf):
        bad = x.copy()
        bad[7, 11, 13] = v
        _, st = O.compress(bad, 1e-3, O.EB_PWREL)
        gst, _, _, _ = gpu_run(bad, 1e-3)
        assert gst == st == O.ERR_NONFINITE
    # a bound whose step is below 2: rejected before any work
    _, st = O.compress(x, 1e-8, O.EB_PWREL)
    assert st == O.ERR_EB_RANGE
    with pytest.raises(fz.FzError) as e:
        fz.compress(torch.from_numpy(x).cuda(), 1e-8, "pwrel")
    assert e.value.code == 4  # FZ_ERR_EB_RANGE, the API code (the stream status bit is O.ERR_EB_RANGE)
    # white noise of random sign: every sign change escapes
    w = np.random.default_rng(9).standard_normal((16, 32, 64)).astype(np.float32)
    _, st = O.compress(w, 1e-3, O.EB_PWREL)
    gst, _, _, _ = gpu_run(w, 1e-3)
    assert gst == st == O.ERR_OUTLIER_CAP


def test_batch_and_server_reject_the_mode():
    """The batched and serving layers take the grid modes only."""
    x = torch.from_numpy(synth.wide_field((20, 40, 70), seed=10)).cuda()
    with pytest.raises(fz.FzError) as e:
        fz.Batch.compress([(x, 1e-3, "pwrel", None)])
    assert e.value.code == 1
    srv = fz.Server(1 << 30)
    try:
        with pytest.raises(fz.FzError) as e:
            srv.submit_compress(x, 1e-3, "pwrel")
        assert e.value.code == 1
    finally:
        srv.close()


@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_full_size_lognormal(eps):
    """512^3 positive values over several binades (the cosmology-like field),
    whole stream and whole reconstruction against the oracle."""
    x = synth.lognormal3d()
    check(x, eps, threads=THREADS)
