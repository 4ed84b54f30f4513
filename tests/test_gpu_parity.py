"""GPU parity: the HIP path against the oracle, through the C ABI.

Streams must be byte-identical and reconstructions bit-identical (the format
fixes one correct stream per input; the floating-point steps use the same
fp32 operation order on both sides).  Sizes span several chunks and ragged
tails; edge cases cover single elements, constant and zero fields, escapes,
and the data-dependent error bits.
"""
import os

import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu


def gpu_compress(x, eb, mode):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    buf = fz.compress(xt, eb, mode="rel" if mode == O.EB_REL else "abs")
    torch.cuda.synchronize()
    n = fz.stream_size(buf)
    return buf, buf[:n].cpu().numpy()


def gpu_decompress(buf, shape):
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, shape, err=err)
    torch.cuda.synchronize()
    return y.cpu().numpy(), int(err.item())


def check_case(x, eb, mode=O.EB_REL):
    print("case", x.shape, eb, mode, flush=True)
    ref, st = O.compress(x, eb, mode)
    buf, s = gpu_compress(x, eb, mode)
    assert st == 0
    assert s.size == ref.size, (s.size, ref.size)
    if not np.array_equal(s, ref):
        diff = np.nonzero(s != ref)[0]
        raise AssertionError("stream differs at %d bytes, first at %d of %d" % (diff.size, diff[0], s.size))
    y, err = gpu_decompress(buf, x.shape)
    assert err == 0
    yo, erro = O.decompress(ref, x.shape)
    assert erro == 0
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))
    return s


CASES = [
    ((64, 64, 64), 0, 1e-3),        # the small 3-D workload
    ((37, 70, 130), 1, 1e-4),       # ragged 3-D, several chunks per dim
    ((16, 32, 64), 2, 1e-2),        # exactly one chunk
    ((17, 33, 65), 3, 1e-3),        # one cell past a chunk in every dim
    ((75, 2050), 4, 1e-3),          # ragged 2-D
    ((32, 1024), 5, 1e-4),          # one 2-D chunk
    ((100000,), 6, 1e-3),           # ragged 1-D
    ((32768 * 3,), 7, 1e-4),        # whole 1-D chunks
    ((5, 3, 2), 8, 1e-3), ((1, 1, 1), 9, 1e-3), ((1,), 10, 1e-3), ((3, 7), 11, 1e-3), ((2, 1, 9000), 12, 1e-3),
]


@pytest.mark.parametrize("shape,seed,eb", CASES)
def test_parity_rel(shape, seed, eb):
    check_case(synth.sine_field(shape, seed=seed), eb)


@pytest.mark.parametrize("shape,seed", [((40, 70, 130), 20), ((70, 2100), 21), ((70001,), 22)])
def test_parity_abs(shape, seed):
    check_case(synth.sine_field(shape, seed=seed), 2.5e-4, O.EB_ABS)


def test_parity_unaligned_width():
    # nx not a multiple of 4 exercises the scalar load/store path
    check_case(synth.sine_field((20, 45, 131), seed=30), 1e-3)
    check_case(synth.sine_field((45, 1027), seed=31), 1e-3)


def test_parity_zero_and_constant_fields():
    check_case(np.zeros((40, 50, 70), np.float32), 1e-3)
    check_case(np.full((40, 50, 70), 3.25, np.float32), 1e-3)
    check_case(np.zeros((100, 1000), np.float32), 1e-3)


def test_parity_escapes():
    x = synth.sine_field((20, 40, 70), seed=2) + np.float32(1000.0)
    s = check_case(x, 1e-3, O.EB_ABS)
    assert fz.stream_info(s[:128].tobytes())["n_outliers"] > 0
    x2 = synth.sine_field((50, 3000), seed=3) + np.float32(500.0)
    check_case(x2, 1e-3, O.EB_ABS)
    x1 = synth.sine_field((70000,), seed=4) + np.float32(500.0)
    check_case(x1, 1e-3, O.EB_ABS)


@pytest.mark.parametrize("shape,count,rows", [
    ((32768,), 150, (0, 8190)),            # 300 escapes in layer 0 of a 1-D chunk
    ((32768,), 129, (8192, 16382)),        # 258 in layer 1
    ((32768,), 512, (16384, 24574)),       # the chunk's whole allowance (1024) in layer 2
    ((16, 32, 64), 40, (4, 7)),            # 3-D, 320 in layer 1 (swept downwards on the fast path)
    ((16, 32, 64), 128, (12, 15)),         # 3-D, 1024 in layer 3
    ((32, 1024), 100, (8, 15)),            # 2-D, 400 in layer 1
    ((33, 70, 130), 300, (4, 7)),          # 3-D, several chunks, edge chunks among them
    ((70, 2100), 400, (40, 47)),           # 2-D, several chunks
])
def test_parity_escapes_crowded_in_one_layer(shape, count, rows):
    """A chunk may hold up to 1024 escapes wherever they fall: layers with
    more than 256 (and up to all 1024) give the oracle's stream."""
    x = synth.spike_field(shape, count, rows, seed=17)
    s = check_case(x, 0.5, O.EB_ABS)
    info = fz.stream_info(s[:128].tobytes())
    assert info["n_outliers"] > 256 and info["status"] == 0


def test_escape_cap_per_chunk_matches_oracle():
    x = synth.spike_field((32768,), 512, (16384, 24574), seed=18)
    x[30000:] = np.float32(100000.0)  # 1025 escapes in one chunk: the cap
    _, st = O.compress(x, 0.5, O.EB_ABS)
    buf, _ = gpu_compress(x, 0.5, O.EB_ABS)
    assert fz.stream_info(buf)["status"] == st == O.ERR_OUTLIER_CAP
    x2 = np.concatenate([synth.spike_field((32768,), 512, (16384, 24574), seed=18), np.zeros(32768, np.float32)])
    x2[40000:] = np.float32(100000.0)  # 1024 + 1 over two chunks: a valid stream
    check_case(x2, 0.5, O.EB_ABS)


def test_status_bits_match_oracle():
    x = synth.sine_field((20, 40, 70), seed=1)
    bad = x.copy()
    bad[3, 4, 5] = np.nan
    for mode in (O.EB_REL, O.EB_ABS):
        _, st = O.compress(bad, 1e-3, mode)
        buf, _ = gpu_compress(bad, 1e-3, mode)
        assert fz.stream_info(buf)["status"] == st == O.ERR_NONFINITE
        _, err = gpu_decompress(buf, bad.shape)
        assert err == 8
    big = x * np.float32(1e30)
    _, st = O.compress(big, 1e-10, O.EB_ABS)
    buf, _ = gpu_compress(big, 1e-10, O.EB_ABS)
    assert fz.stream_info(buf)["status"] == st == O.ERR_EB_RANGE
    rng = np.random.default_rng(3)
    w = (rng.standard_normal((16, 32, 64)) * 1e6).astype(np.float32)
    _, st = O.compress(w, 0.5, O.EB_ABS)
    buf, _ = gpu_compress(w, 0.5, O.EB_ABS)
    assert fz.stream_info(buf)["status"] == st == O.ERR_OUTLIER_CAP


def test_status_precedence():
    """NaN / Inf or an overflowing x/(2eb) end the pipeline at
    prequantization: the escape-cap bit, which the rest of the field alone
    would set, is not reported with them."""
    rng = np.random.default_rng(4)
    w = (rng.standard_normal((20, 40, 70)) * 1e6).astype(np.float32)
    for v, eb, want in ((np.nan, 0.5, O.ERR_NONFINITE), (np.inf, 0.5, O.ERR_NONFINITE),
                        (np.float32(3e38), 0.5, O.ERR_EB_RANGE)):
        bad = w.copy()
        bad[19, 39, 69] = v
        _, st = O.compress(bad, eb, O.EB_ABS)
        buf, _ = gpu_compress(bad, eb, O.EB_ABS)
        assert fz.stream_info(buf)["status"] == st == want


@pytest.mark.parametrize("where", [(0, 0, 0), (63, 511, 1023), (40, 300, 700)])
def test_status_precedence_full_grid(where):
    """The same on 1024 chunks, more than the persistent grid has
    workgroups: every chunk holds more escapes than the cap allows, and one
    chunk also a NaN.  The grid's last workgroup to finish settles the status
    word, whichever workgroups set its bits, so the escape-cap bit is never
    reported with NONFINITE."""
    rng = np.random.default_rng(6)
    w = (rng.standard_normal((64, 512, 1024)) * 1e6).astype(np.float32)
    w[where] = np.nan
    print("full-grid precedence", where, flush=True)
    _, st = O.compress(w, 0.5, O.EB_ABS, threads=min(os.cpu_count() or 1, 16))
    buf, _ = gpu_compress(w, 0.5, O.EB_ABS)
    assert fz.stream_info(buf)["status"] == st == O.ERR_NONFINITE
    w[where] = 0.0
    _, st = O.compress(w, 0.5, O.EB_ABS, threads=min(os.cpu_count() or 1, 16))
    buf, _ = gpu_compress(w, 0.5, O.EB_ABS)
    assert fz.stream_info(buf)["status"] == st == O.ERR_OUTLIER_CAP


@pytest.mark.parametrize("where", ["first", "last", "tail", "middle"])
@pytest.mark.parametrize("val", [np.inf, -np.inf, np.nan])
def test_rel_range_nonfinite(where, val):
    """A NaN or an infinity anywhere (also among the last values that do not
    fill a 16-byte vector) fails the REL range pass, as in the oracle (the
    rest of a failed stream is unspecified)."""
    x = synth.sine_field((100003,), seed=11)  # n % 4 == 3: a scalar tail
    i = {"first": 0, "last": x.size - 1, "tail": x.size - 2, "middle": 51234}[where]
    x[i] = val
    print("nonfinite", where, val, flush=True)
    _, st = O.compress(x, 1e-3, O.EB_REL)
    buf, s = gpu_compress(x, 1e-3, O.EB_REL)
    assert fz.stream_info(buf)["status"] == st == O.ERR_NONFINITE


def test_rel_range_signed_zero_and_constant():
    """The range pass on signed zeros and constant fields gives the oracle's
    header (vmin / vmax, eb) and stream."""
    x = synth.sine_field((20, 40, 70), seed=12)
    x[x < 0] = np.float32(-0.0)  # minimum -0.0, all others >= 0
    check_case(x, 1e-3)
    check_case(np.full((33, 1030), -0.0, dtype=np.float32), 1e-3)
    check_case(np.full((70001,), -2.5, dtype=np.float32), 1e-3)


def test_decompress_rejects_bad_stream():
    x = synth.sine_field((20, 40, 70), seed=5)
    buf, s = gpu_compress(x, 1e-3, O.EB_REL)
    bad = buf.clone()
    bad[0] = 0
    _, err = gpu_decompress(bad, x.shape)
    assert err == 6
    bad = buf.clone()
    bad[4] = 9
    _, err = gpu_decompress(bad, x.shape)
    assert err == 7
    _, err = gpu_decompress(buf, (20, 40, 71))
    assert err == 6


def test_decompress_bounds_and_table_checks():
    """The device reads no byte past stream_bytes and checks the chunk table
    against the flags: a stream cut short (in a buffer of exactly the cut
    length), a total beyond the buffer, a table offset moved by one unit, and
    a flag bit set without its brick are all rejected with FZ_ERR_STREAM;
    the intact stream in an exact-size buffer decodes."""
    x = synth.sine_field((40, 70, 130), seed=8)  # 24 chunks
    buf, s = gpu_compress(x, 1e-3, O.EB_REL)
    exact = torch.from_numpy(s.copy()).cuda()
    y, err = gpu_decompress(exact, x.shape)
    yo, _ = O.decompress(s, x.shape)
    assert err == 0 and np.array_equal(y.view(np.uint32), yo.view(np.uint32))
    hb = fz.header_bytes(x.shape)
    for cut in (hb, hb + 16, (hb + s.size) // 2, s.size - 16):
        short = torch.from_numpy(s[:cut].copy()).cuda()
        _, err = gpu_decompress(short, x.shape)
        assert err == 6, cut
    nch = fz.stream_info(s[:128].tobytes())["n_chunks"]
    for c in (1, nch // 2, nch - 1):  # chunk c's offset, one unit later
        t = s.copy()
        tab = t[128:128 + 8 * nch].view(np.uint32).reshape(nch, 2)
        tab[c, 0] += 1
        _, err = gpu_decompress(torch.from_numpy(t).cuda(), x.shape)
        assert err == 6, c
    t = s.copy()
    flags = t[hb - 512 * nch:hb].view(np.uint64)
    zero = np.nonzero(flags[:64] != np.uint64(0xFFFFFFFFFFFFFFFF))[0][0]  # a flag word of chunk 0 with a free bit
    free = [b for b in range(64) if not (int(flags[zero]) >> b) & 1][0]
    flags[zero] |= np.uint64(1) << np.uint64(free)
    _, err = gpu_decompress(torch.from_numpy(t).cuda(), x.shape)
    assert err == 6


def test_deterministic_repeats():
    x = synth.sine_field((48, 96, 200), seed=6)
    _, a = gpu_compress(x, 1e-4, O.EB_REL)
    for _ in range(5):
        _, b = gpu_compress(x, 1e-4, O.EB_REL)
        assert np.array_equal(a, b)
