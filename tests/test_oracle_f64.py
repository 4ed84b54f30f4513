"""Pins of the oracle's fp64 input path (CPU only).

The fp64 path quantizes in double precision (q = rint(x * inv), inv = 1 /
(2 eb_abs)) and feeds the same integer encoder as the fp32 path.  The pins:
integer-valued fields at eb = 1/2 give the fp32 stream's payload byte for
byte and reproduce the input exactly; the independent numpy stream reader
reads back the integers; the textbook bound |x' - x| <= eb (Sec. 2.3) holds
on round trips, also for values closer together than fp32 can tell apart;
ties round to even; the value range of REL mode is taken in double; and the
statuses (non-finite input, an unusable bound, x / (2 eb) beyond int32).
"""
import numpy as np
import pytest

from oracle import oracle as O
import stream_np
import synth


def test_integer_field_matches_the_fp32_stream():
    rng = np.random.default_rng(1)
    x = np.cumsum(rng.integers(-3, 4, size=(20, 40, 70)), axis=2).astype(np.float64)
    s64, st64 = O.compress_f64(x, 0.5, O.EB_ABS)
    s32, st32 = O.compress(x.astype(np.float32), 0.5, O.EB_ABS)
    assert st64 == st32 == 0 and s64.size == s32.size
    diff = np.nonzero(s64 != s32)[0]
    # only the dtype byte and the fp64 bound parameters differ
    assert set(diff.tolist()) <= {12} | set(range(104, 120))
    assert s64[12] == 1 and s32[12] == 0
    assert np.frombuffer(s64[104:112].tobytes(), np.float64)[0] == 1.0
    assert np.frombuffer(s64[112:120].tobytes(), np.float64)[0] == 1.0
    y, err = O.decompress_f64(s64, x.shape)
    assert err == 0 and np.array_equal(y, x)


@pytest.mark.parametrize("shape,eb,mode", [((20, 40, 70), 1e-4, O.EB_REL), ((45, 1030), 1e-3, O.EB_ABS),
                                           ((70001,), 1e-5, O.EB_REL)])
def test_round_trip_bound_and_reader(shape, eb, mode):
    x = synth.sine_field(shape, seed=sum(shape)).astype(np.float64) * 1.000000123
    s, st = O.compress_f64(x, eb, mode)
    assert st == 0
    h = stream_np.header(s)
    assert h["dtype"] == 1
    ebx2 = np.frombuffer(s[104:112].tobytes(), np.float64)[0]
    inv = np.frombuffer(s[112:120].tobytes(), np.float64)[0]
    eb_abs = eb if mode == O.EB_ABS else eb * (x.max() - x.min())
    assert ebx2 == 2.0 * eb_abs and inv == 1.0 / ebx2
    q = stream_np.read(s, shape)["q"]
    assert np.array_equal(q, np.rint(x * inv).astype(np.int32))
    y, err = O.decompress_f64(s, shape)
    assert err == 0
    assert np.all(np.abs(y - x) <= eb_abs * (1 + 2.0 ** -40))


def test_precision_beyond_fp32():
    # values 2^-44 apart near 2^-16 (fp32 keeps one in 32 apart) with a bound
    # of 2^-46 (q near 2^29)
    k = np.arange(4096, dtype=np.float64)
    x = 2.0 ** -16 + k * 2.0 ** -44
    assert np.unique(x.astype(np.float32)).size <= x.size // 32 + 1
    s, st = O.compress_f64(x, 2.0 ** -46, O.EB_ABS)
    assert st == 0
    y, err = O.decompress_f64(s, x.shape)
    assert err == 0 and np.all(np.abs(y - x) <= 2.0 ** -46)
    assert np.unique(y).size == x.size


def test_ties_round_to_even():
    x = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 3.5, 1e6 + 0.5], dtype=np.float64)
    q, st = O.prequant_f64(x, 1.0)
    assert st == 0
    assert q.tolist() == [0, 2, 2, 0, -2, -2, 4, 1000000]


def test_rel_range_in_double():
    x = np.full((3, 4, 5), 1e10)
    x[1, 2, 3] = 1e10 + 1.0  # fp32 cannot tell the two apart
    p = O.eb_params_f64(x, 1e-3, O.EB_REL)
    assert p["status"] == 0 and p["vmin"] == 1e10 and p["vmax"] == 1e10 + 1.0
    assert p["ebx2"] == 2.0 * (1e-3 * 1.0)
    # constant and all-zero fields
    assert O.eb_params_f64(np.full(7, -4.0), 1e-2, O.EB_REL)["ebx2"] == 2.0 * (1e-2 * 4.0)
    assert O.eb_params_f64(np.zeros(7), 1e-2, O.EB_REL)["ebx2"] == 2.0 * 1e-2
    # -0 counts as +0 in the range
    p = O.eb_params_f64(np.array([-0.0, 2.0]), 0.25, O.EB_REL)
    assert p["vmin"] == 0.0 and not np.signbit(p["vmin"]) and p["ebx2"] == 1.0


def test_statuses():
    x = synth.sine_field((20, 40, 70), seed=3).astype(np.float64)
    for v in (np.nan, np.inf, -np.inf):
        bad = x.copy()
        bad[3, 4, 5] = v
        for mode in (O.EB_ABS, O.EB_REL):
            assert O.compress_f64(bad, 1e-3, mode)[1] == O.ERR_NONFINITE
    assert O.compress_f64(x, 1e-310, O.EB_ABS)[1] == O.ERR_EB_RANGE  # 2 eb below the smallest normal double
    big = x * 1e30
    assert O.compress_f64(big, 1e-3, O.EB_ABS)[1] == O.ERR_EB_RANGE  # |x / (2 eb)| >= 2^31
    with pytest.raises(ValueError):
        O.compress_f64(x, 1e-3, O.EB_PWREL)  # the point-wise mode takes fp32 input only


def test_streams_of_one_type_do_not_decode_as_the_other():
    x = synth.sine_field((16, 32, 64), seed=4)
    s32, _ = O.compress(x, 1e-3, O.EB_REL)
    s64, _ = O.compress_f64(x.astype(np.float64), 1e-3, O.EB_REL)
    assert O.decompress_f64(s32, x.shape)[1] != 0
    assert O.decompress(s64, x.shape)[1] != 0


def test_large_values_with_a_small_bound():
    # q near 5e8: fp32 bound parameters or an fp32 product would miss the
    # bound by far (fp32 spacing at 1e6 is 0.0625)
    x = 1e6 + synth.sine_field((20, 40, 70), seed=5).astype(np.float64) * 10.0
    s, st = O.compress_f64(x, 1e-3, O.EB_ABS)
    assert st == 0
    y, err = O.decompress_f64(s, x.shape)
    assert err == 0 and np.all(np.abs(y - x) <= 1e-3 * (1 + 2.0 ** -40))
