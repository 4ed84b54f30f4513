"""The distortion pass on the GPU against the oracle, through the C ABI.

The maximum difference, the value range, n and the non-finite count are
order-independent and must match the oracle exactly.  The MSE is a sum of n
doubles in another order: each partial sum is rounded at most once per
addition, so the relative difference is below n * 2^-53; the test allows
1e-12 for the sizes here (and 1e-9 at 512^3).  PSNR inherits that through
the logarithm (absolute dB difference below 1e-9).
"""
import math

import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import quality as Q
import synth

pytestmark = pytest.mark.gpu


def check(x, y, rel=1e-12):
    q = fz.quality(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    r = Q.quality(x, y)
    for k in ("n", "nonfinite"):
        assert q[k] == r[k], k
    if r["nonfinite"]:
        assert all(math.isnan(q[k]) for k in ("max_abs_err", "mse", "psnr", "vmin", "vmax"))
        return q
    for k in ("max_abs_err", "vmin", "vmax"):
        assert q[k] == r[k], (k, q[k], r[k])
    assert q["mse"] == pytest.approx(r["mse"], rel=rel)
    if math.isinf(r["psnr"]):
        assert q["psnr"] == r["psnr"]
    else:
        assert abs(q["psnr"] - r["psnr"]) < 1e-9
    return q


@pytest.mark.parametrize("shape", [(1,), (3,), (1000,), (1000003,), (37, 70, 130), (75, 2050), (64, 64, 64),
                                   (3, 1, 5)])
def test_random_fields(shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape).astype(np.float32) * np.float32(3.0)
    y = (x + rng.standard_normal(shape).astype(np.float32) * np.float32(1e-3)).astype(np.float32)
    print("quality", shape, flush=True)
    check(x, y)


def test_unaligned_rows_take_the_scalar_path():
    rng = np.random.default_rng(5)
    xt = torch.from_numpy(rng.standard_normal(100001).astype(np.float32)).cuda()
    yt = xt + 1e-3 * torch.randn(100001, device="cuda")
    x, y = xt[1:], yt[1:].contiguous()  # x starts 4 bytes into its allocation
    q = fz.quality(x, y)
    r = Q.quality(x.cpu().numpy(), y.cpu().numpy())
    assert q["max_abs_err"] == r["max_abs_err"] and q["vmin"] == r["vmin"] and q["vmax"] == r["vmax"]
    assert q["mse"] == pytest.approx(r["mse"], rel=1e-12)


def test_identical_and_constant():
    x = np.full((20, 30), 2.5, dtype=np.float32)
    assert check(x, x.copy())["psnr"] == math.inf
    assert check(x, x + np.float32(1.0))["psnr"] == -math.inf


@pytest.mark.parametrize("where", [0, 4095, 99998, 50000])
@pytest.mark.parametrize("val", [np.nan, np.inf])
def test_nonfinite(where, val):
    x = synth.sine_field((99999,), seed=8)  # n % 4 == 3: a scalar tail
    y = x.copy()
    y[where] = val
    check(x, y)


def test_round_trip_respects_the_bound_and_is_deterministic():
    x = synth.sine_field((64, 64, 64), seed=0)
    xt = torch.from_numpy(x).cuda()
    s = fz.compress(xt, 1e-3, "rel")
    y = fz.decompress(s, x.shape)
    info = fz.stream_info(s)
    eb_abs = 1e-3 * (float(info["vmax"]) - float(info["vmin"]))
    q = check(x, y.cpu().numpy())
    # the bound holds up to fp32 rounding of x / (2 eb) and of q * 2 eb: an ulp or two of the values
    slack = 4 * float(np.spacing(np.float32(np.abs(x).max())))
    assert 0 < q["max_abs_err"] <= eb_abs + slack
    q2 = fz.quality(xt, y)
    assert all(q[k] == q2[k] for k in q)  # the same bits on a second call
