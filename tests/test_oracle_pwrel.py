"""Pins of the oracle's point-wise relative mode (CPU only).

The mode compresses the float's bit pattern (a piecewise-linear log2, exact
in integers) with the absolute step S that the relative bound implies.  The
pins check the step formula, closed forms at powers of two, symmetry in the
sign, zeros, the largest float, brute-force integer quantization, and the
point-wise bound |x' - x| <= eps * max(|x|, 2^-126) on whole round trips over
fields spanning many binades, with sign changes (escapes) and denormals.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
import synth

FLT_MIN = 2.0 ** -126


def step_of(eps):
    p = O.eb_params(np.zeros(4, np.float32), eps, O.EB_PWREL)
    return int(p["ebx2"]), p["status"]


def test_step_formula():
    assert step_of(1e-3) == (math.floor(1e-3 * 2 ** 24 / 1.001), 0) == (16760, 0)
    assert step_of(0.5) == (5592405, 0)
    assert step_of(1.2e-7) == (2, 0)
    assert step_of(1.1e-7)[1] == O.ERR_EB_RANGE  # S < 2
    # the step grows with the bound
    steps = [step_of(e)[0] for e in (1e-6, 1e-4, 1e-2, 0.1, 0.9, 5.0)]
    assert steps == sorted(steps) and steps[-1] < 2 ** 24


def test_powers_of_two_are_exact_when_the_step_divides_the_binade():
    x = np.array([2.0 ** k for k in range(-126, 128, 7)], dtype=np.float32)
    q, st = O.prequant_pw(x, 8192)
    assert st == 0
    b = x.view(np.uint32).astype(np.int64)
    assert np.array_equal(q, b // 8192)  # b is a multiple of 2^23
    assert all(O.dequant_pw(int(v), 8192) == xv for v, xv in zip(q, x))


def test_sign_symmetry_zero_and_extremes():
    x = np.array([1.5, -1.5, 0.0, -0.0, 3.4028235e38, -3.4028235e38, 1e-40, -1e-40], dtype=np.float32)
    q, st = O.prequant_pw(x, 16760)
    assert st == 0
    assert q[0] == -q[1] and q[4] == -q[5] and q[6] == -q[7]
    assert q[2] == 0 and q[3] == 0
    assert O.dequant_pw(0, 16760) == 0.0 and math.copysign(1.0, O.dequant_pw(0, 16760)) == 1.0
    big = O.dequant_pw(int(q[4]), 16760)
    assert np.isfinite(big) and big <= np.float32(3.4028235e38)  # clamped to the largest float
    assert O.dequant_pw(int(q[1]), 16760) < 0


def test_nonfinite_input():
    for v in (np.nan, np.inf, -np.inf):
        _, st = O.prequant_pw(np.array([1.0, v], np.float32), 100)
        assert st == O.ERR_NONFINITE


@pytest.mark.parametrize("step", [2, 3, 1000, 16760, 5592405, 2 ** 24 - 1])
def test_quantization_brute_force(step):
    rng = np.random.default_rng(step)
    bits = rng.integers(0, 0x7F800000, size=2000, dtype=np.int64)
    sign = rng.integers(0, 2, size=2000, dtype=np.int64)
    x = (bits | (sign << 31)).astype(np.uint32).view(np.float32)
    q, st = O.prequant_pw(x, step)
    assert st == 0
    for i in range(0, 2000, 7):
        a = (int(bits[i]) + step // 2) // step
        assert q[i] == (-a if sign[i] else a)
        m = min(a * step, 0x7F7FFFFF)
        assert abs(m - int(bits[i])) <= step // 2 + (1 if m == 0x7F7FFFFF else 0) or m == 0x7F7FFFFF


@pytest.mark.parametrize("shape,eps", [((20, 40, 70), 1e-3), ((45, 1030), 1e-2), ((70001,), 1e-4),
                                       ((16, 32, 64), 0.3)])
def test_round_trip_point_wise_bound(shape, eps):
    x = synth.wide_field(shape, seed=sum(shape))
    s, st = O.compress(x, eps, O.EB_PWREL)
    assert st == 0
    y, err = O.decompress(s, shape)
    assert err == 0
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    allowed = eps * np.maximum(np.abs(xd), FLT_MIN)
    assert np.all(np.abs(yd - xd) <= allowed)
    assert np.all((yd < 0) == (xd < 0))  # signs kept (zeros come back +0)
    assert np.all(y[x == 0] == 0)
