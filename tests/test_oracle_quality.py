"""Pins of the distortion-metric oracle (CPU only).

Closed forms, special cases and brute force on tiny inputs, chosen so that a
plausible mistake fails one of them: a difference taken in fp32 instead of
double, the reconstruction's range instead of the original's, RMSE for MSE,
a missing non-finite check, or a wrong sign in the PSNR terms.
"""
import math

import numpy as np
import pytest

from oracle import quality as Q


def test_identical_fields():
    x = np.linspace(-3, 5, 1001, dtype=np.float32)
    q = Q.quality(x, x)
    assert q["max_abs_err"] == 0.0 and q["mse"] == 0.0 and q["psnr"] == math.inf
    assert q["vmin"] == -3.0 and q["vmax"] == 5.0 and q["n"] == 1001 and q["nonfinite"] == 0


def test_constant_shift_closed_form():
    x = np.arange(1000, dtype=np.float32)
    y = x + np.float32(0.25)  # exact in fp32 below 2^22
    q = Q.quality(x, y)
    assert q["max_abs_err"] == 0.25
    assert q["mse"] == 0.0625
    assert q["psnr"] == pytest.approx(20 * math.log10(999.0) - 10 * math.log10(0.0625), rel=1e-15)


def test_range_is_the_originals_and_mse_not_rmse():
    x = np.array([0, 1, 2, 3, 4], dtype=np.float32)
    y = np.zeros(5, dtype=np.float32)  # its own range is 0
    q = Q.quality(x, y)
    assert q["max_abs_err"] == 4.0
    assert q["mse"] == 6.0  # (0 + 1 + 4 + 9 + 16) / 5
    assert q["psnr"] == pytest.approx(20 * math.log10(4.0) - 10 * math.log10(6.0), rel=1e-15)


def test_difference_taken_in_double():
    x = np.array([1.0], dtype=np.float32)
    y = np.array([2.0 ** -30], dtype=np.float32)  # 1 - 2^-30 rounds to 1 in fp32
    q = Q.quality(x, y)
    assert q["max_abs_err"] == 1.0 - 2.0 ** -30


def test_constant_original():
    x = np.full(10, 3.0, dtype=np.float32)
    assert Q.quality(x, x)["psnr"] == math.inf
    assert Q.quality(x, x + np.float32(1.0))["psnr"] == -math.inf


@pytest.mark.parametrize("where,val", [(0, np.nan), (7, np.inf), (12, -np.inf)])
@pytest.mark.parametrize("side", ["x", "y"])
def test_nonfinite(where, val, side):
    x = np.linspace(0, 1, 13, dtype=np.float32)
    y = x.copy()
    (x if side == "x" else y)[where] = val
    q = Q.quality(x, y)
    assert q["nonfinite"] == 1 and q["n"] == 13
    assert all(math.isnan(q[k]) for k in ("max_abs_err", "mse", "psnr", "vmin", "vmax"))


@pytest.mark.parametrize("seed", range(20))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    x = (rng.standard_normal(n) * 10 ** rng.uniform(-3, 3)).astype(np.float32)
    y = (x + rng.standard_normal(n).astype(np.float32) * np.float32(1e-2)).astype(np.float32)
    e = [float(a) - float(b) for a, b in zip(x.tolist(), y.tolist())]
    mse = math.fsum(v * v for v in e) / n
    q = Q.quality(x, y)
    assert q["max_abs_err"] == max(abs(v) for v in e)
    assert q["mse"] == pytest.approx(mse, rel=1e-14)
    assert q["vmin"] == min(x.tolist()) and q["vmax"] == max(x.tolist())
    rng_ = max(x.tolist()) - min(x.tolist())
    if mse > 0 and rng_ > 0:
        assert q["psnr"] == pytest.approx(20 * math.log10(rng_) - 10 * math.log10(mse), rel=1e-13)


def test_bitrate_and_overall_throughput():
    assert Q.bitrate(10.0) == 3.2  # 32 bits over the ratio
    assert Q.bitrate(1.0) == 32.0
    # equal link-side (bw * ratio) and compression rates halve the throughput
    assert Q.overall_throughput(10.0, 10.0, 100.0) == pytest.approx(50.0, rel=1e-15)
    # an infinitely fast compressor leaves the link at bw * ratio
    assert Q.overall_throughput(11.4, 20.0, 1e300) == pytest.approx(228.0, rel=1e-12)
    # an infinitely fast link leaves the compressor
    assert Q.overall_throughput(1e300, 5.0, 1700.0) == pytest.approx(1700.0, rel=1e-12)
