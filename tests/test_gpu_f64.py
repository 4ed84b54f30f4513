"""GPU parity of the fp64 input path (fz_compress_f64 / fz_decompress_f64)
through the C ABI.

The bar is that of the fp32 parity tests: the oracle's status, and when it
is 0 the same stream bytes and the same reconstruction bits.  Cases: the
three ranks with whole and ragged chunk boxes, contiguous extents that are
not multiples of 4, an input pointer that is 8- but not 16-byte aligned (the
scalar loads of the range and prequantization passes), values closer
together than fp32 can tell apart, large magnitudes with a small bound, the
statuses and their precedence, streams of the other type, and the whole
hurricane-like field.
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


def field64(shape, seed):
    return synth.sine_field(shape, seed=seed).astype(np.float64) * 1.000000123


def gpu_run(x, eb, mode, misalign=False):
    if misalign:  # 8-byte aligned only: one double in front
        big = torch.empty(x.size + 1, dtype=torch.float64, device="cuda")
        xt = big[1:].view(x.shape)
        xt.copy_(torch.from_numpy(x))
    else:
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    buf = fz.compress(xt, eb, "rel" if mode == O.EB_REL else "abs")
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    if info["status"]:
        return info["status"], None, None, None
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, x.shape, err=err, dtype=torch.float64)
    torch.cuda.synchronize()
    n = int(info["total_bytes"])
    return 0, buf[:n].cpu().numpy(), y.cpu().numpy(), int(err.item())


def check(x, eb, mode, threads=1, misalign=False):
    print("f64 case", x.shape, eb, mode, misalign, flush=True)
    ref, st = O.compress_f64(x, eb, mode, threads=threads)
    gst, s, y, err = gpu_run(x, eb, mode, misalign)
    assert gst == st == 0, (gst, st)
    assert s.size == ref.size, (s.size, ref.size)
    if not np.array_equal(s, ref):
        diff = np.nonzero(s != ref)[0]
        raise AssertionError("stream differs at %d bytes, first at %d of %d" % (diff.size, diff[0], s.size))
    assert err == 0
    yo, erro = O.decompress_f64(ref, x.shape)
    assert erro == 0
    assert np.array_equal(y.view(np.uint64), yo.view(np.uint64))
    return s, y


@pytest.mark.parametrize("shape,eb,mode", [
    ((20, 40, 70), 1e-4, O.EB_REL),    # 3-D, ragged in every dimension
    ((16, 32, 64), 1e-3, O.EB_ABS),    # one whole chunk box
    ((33, 65, 131), 1e-3, O.EB_REL),   # box + 1, contiguous extent odd
    ((45, 1030), 1e-3, O.EB_ABS),      # 2-D ragged
    ((33, 1027), 1e-4, O.EB_REL),      # 2-D, contiguous extent not a multiple of 4
    ((70, 2052), 1e-4, O.EB_REL),      # 2-D, 3 x 3 chunks, whole rows through the LDS tile
    ((40, 70, 128), 1e-3, O.EB_ABS),   # 3-D, interior chunks through the LDS tile
    ((70001,), 1e-5, O.EB_REL),        # 1-D ragged
    ((65537,), 1e-3, O.EB_ABS),        # 1-D, two chunks and one value
    ((1,), 1e-3, O.EB_REL), ((3, 1, 5), 1e-3, O.EB_ABS),
])
def test_parity(shape, eb, mode):
    check(field64(shape, sum(shape)), eb, mode)


@pytest.mark.parametrize("shape", [(20, 40, 70), (70001,), (45, 1031)])
def test_misaligned_input(shape):
    check(field64(shape, 7 + sum(shape)), 1e-4, O.EB_REL, misalign=True)


def test_precision_beyond_fp32_and_large_values():
    k = np.arange(4096, dtype=np.float64)
    _, y = check(2.0 ** -16 + k * 2.0 ** -44, 2.0 ** -46, O.EB_ABS)
    assert np.unique(y).size == k.size
    x = 1e6 + field64((20, 40, 70), 5) * 10.0
    _, y = check(x, 1e-3, O.EB_ABS)
    assert np.all(np.abs(y - x) <= 1e-3 * (1 + 2.0 ** -40))


def test_statuses_and_precedence():
    x = field64((20, 40, 70), 3)
    for v in (np.nan, np.inf, -np.inf):
        bad = x.copy()
        bad[3, 4, 5] = v
        for mode in (O.EB_ABS, O.EB_REL):
            _, st = O.compress_f64(bad, 1e-3, mode)
            assert gpu_run(bad, 1e-3, mode)[0] == st == O.ERR_NONFINITE
    big = x * 1e30
    _, st = O.compress_f64(big, 1e-3, O.EB_ABS)
    assert gpu_run(big, 1e-3, O.EB_ABS)[0] == st == O.ERR_EB_RANGE
    with pytest.raises(fz.FzError) as e:
        fz.compress(torch.from_numpy(x).cuda(), 1e-310, "abs")
    assert e.value.code == 4  # FZ_ERR_EB_RANGE, before any work
    with pytest.raises(fz.FzError) as e:
        fz.compress(torch.from_numpy(x).cuda(), 1e-3, "pwrel")
    assert e.value.code == 1
    noise = np.random.default_rng(4).standard_normal((20, 40, 70)) * 1e6
    _, st = O.compress_f64(noise, 0.5, O.EB_ABS)
    assert gpu_run(noise, 0.5, O.EB_ABS)[0] == st == O.ERR_OUTLIER_CAP
    noise[19, 39, 69] = np.nan  # prequantization fails first: its bit alone
    _, st = O.compress_f64(noise, 0.5, O.EB_ABS)
    assert gpu_run(noise, 0.5, O.EB_ABS)[0] == st == O.ERR_NONFINITE


def test_streams_of_the_other_type_are_rejected():
    x = synth.sine_field((16, 32, 64), seed=9)
    s32 = fz.compress(torch.from_numpy(x).cuda(), 1e-3, "rel")
    s64 = fz.compress(torch.from_numpy(x.astype(np.float64)).cuda(), 1e-3, "rel")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    fz.decompress(s32, x.shape, err=err, dtype=torch.float64)
    torch.cuda.synchronize()
    assert int(err.item()) == 6
    fz.decompress(s64, x.shape, err=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 6
    info = fz.stream_info(s64)
    assert info["dtype"] == 1 and info["ebx2_f64"] > 0 and fz.stream_info(s32)["dtype"] == 0


def test_full_size_hurricane():
    """100 x 500 x 500 in fp64, REL 1e-4: whole stream and reconstruction."""
    x = synth.hurricane3d().astype(np.float64)
    check(x, 1e-4, O.EB_REL, threads=THREADS)
