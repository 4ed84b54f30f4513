"""Pins of the oracle against facts that do not come from the oracle itself.

Each test checks the oracle (``oracle/fzo.c``) against something the paper or
mathematics fixes: the pointwise prequantization of Sec. 2.3 recomputed with
numpy float32, the error-bound inequality of Sec. 2.3, the exact inverse of the
Lorenzo predictor (prefix sums, computed here with numpy cumsum), the
annihilation of lower-dimensional functions by the Lorenzo difference, the
sign-magnitude code of Sec. 3.2 checked exhaustively, bit-count invariants of
the bitshuffle, the size identity of the zero-block encoder (Sec. 3.4), and a
hand-worked example.  A dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle makes at least one of them fail.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
import stream_np
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _q_numpy(x, inv):
    p = np.float32(x) * np.float32(inv)
    return np.rint(p).astype(np.int32)


# ------------------------------------------------------------ prequantization
@pytest.mark.parametrize("scale", [1e-30, 1e-3, 1.0, 1e6])
def test_prequant_matches_pointwise_definition(scale):
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * scale).astype(np.float32)
    eb = 1e-3 * scale
    prm = O.eb_params(x, eb, O.EB_ABS)
    q, st = O.prequant(x, prm["inv"])
    assert st == 0
    assert np.array_equal(q, _q_numpy(x, prm["inv"]))


def test_prequant_ties_round_to_even():
    inv = np.float32(1.0)
    x = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 3.5, 1e6 + 0.5], np.float32)
    q, st = O.prequant(x, inv)
    assert st == 0
    assert q.tolist() == [0, 2, 2, 0, -2, -2, 4, 1000000]


def test_prequant_denormals_are_not_flushed():
    # 0.75 * 2^-126 is subnormal; times 2^127 it is 1.5 -> 2 (half-even).
    # A flush-to-zero multiply would give 0.
    x = np.array([np.float32(2.0 ** -126) * np.float32(0.75), np.float32(2.0 ** -149)], np.float32)
    q, st = O.prequant(x, np.float32(2.0 ** 127))
    assert st == 0 and q.tolist() == [2, 0]
    # subnormal inputs whose products with a finite inv = 2^127 are exactly
    # 0.5, 1.5, -1.5, 1.25 and 1.75 (half-even: 0, 2, -2; nearest: 1, 2),
    # and 2^-149 * 2^127 = 2^-22 -> 0
    inv = np.float32(2.0 ** 127)
    assert np.isfinite(inv)
    x = np.array([2.0 ** -128, 3 * 2.0 ** -128, -3 * 2.0 ** -128, 5 * 2.0 ** -129, 7 * 2.0 ** -129, 2.0 ** -149],
                 np.float32)
    assert np.all(np.abs(x) < np.float32(2.0 ** -126))  # all subnormal
    q, st = O.prequant(x, inv)
    assert st == 0 and q.tolist() == [0, 2, -2, 1, 2, 0]


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_reconstruction_error_bound(rel):
    x = synth.sine_field((40, 37, 70), seed=7)
    s, st = O.compress(x, rel, O.EB_REL)
    assert st == 0
    y, err = O.decompress(s, x.shape)
    assert err == 0
    rng = float(x.max()) - float(x.min())
    eb_abs = rel * rng
    h = stream_np.header(s)
    ebx2 = float(h["ebx2"])
    e = np.abs(x.astype(np.float64) - y.astype(np.float64))
    # provable bound: half the grid step, plus the fp32 rounding of x*inv and of q*ebx2
    bound = ebx2 / 2 + np.abs(x) * 2.0 ** -23 + np.abs(y) * 2.0 ** -24 + 1e-45
    assert np.all(e <= bound)
    # the paper's bound eb (Sec. 2.3) up to a couple of ulps
    ulp = np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)
    assert np.all(e <= eb_abs * (1 + 2.0 ** -23) + 2 * ulp + np.spacing(np.abs(y)).astype(np.float64))


def test_reconstruction_equals_closed_form():
    """decompress(compress(x)) == fp32(rint(x*inv) * ebx2): the lossless stages
    must be exactly invertible, so this pins every stage at once."""
    for shape, seed in [((33, 65, 130), 3), ((97, 1100), 4), ((70001,), 5), ((17, 1, 5), 6)]:
        x = synth.sine_field(shape, seed=seed)
        s, st = O.compress(x, 1e-4, O.EB_REL)
        assert st == 0
        y, err = O.decompress(s, x.shape)
        assert err == 0
        h = stream_np.header(s)
        ref = _q_numpy(x, h["inv"]).astype(np.float32) * np.float32(h["ebx2"])
        assert np.array_equal(y.view(np.uint32), ref.view(np.uint32))


# ------------------------------------------------------------------- Lorenzo
def _chunk_prefix(delta, rank):
    box = stream_np.BOX[rank]
    out = np.zeros(delta.shape, dtype=np.uint32)
    grid = [range(0, delta.shape[i], box[i]) for i in range(rank)]
    import itertools
    for org in itertools.product(*grid):
        sl = tuple(slice(org[i], org[i] + box[i]) for i in range(rank))
        B = delta[sl].astype(np.int64).astype(np.uint32)
        for ax in range(rank):
            B = np.cumsum(B, axis=ax, dtype=np.uint32)
        out[sl] = B
    return out.view(np.int32)


@pytest.mark.parametrize("shape", [(40, 70, 130), (70, 2100), (70000,), (3, 5, 7), (1, 1, 1)])
def test_lorenzo_prefix_sum_is_exact_inverse(shape):
    rng = np.random.default_rng(11)
    q = rng.integers(-(2 ** 31), 2 ** 31, size=shape, dtype=np.int64).astype(np.int32)
    d = O.lorenzo_field(q)
    assert np.array_equal(_chunk_prefix(d, len(shape)), q)


def test_lorenzo_annihilates_lower_dimensional_sums():
    rng = np.random.default_rng(12)
    Z, Y, X = 20, 40, 70
    A = rng.integers(-1000, 1000, size=(Z, Y, 1))
    B = rng.integers(-1000, 1000, size=(Z, 1, X))
    C = rng.integers(-1000, 1000, size=(1, Y, X))
    q = (A + B + C).astype(np.int32)
    d = O.lorenzo_field(q)
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    interior = (z % 16 > 0) & (y % 32 > 0) & (x % 64 > 0)
    assert np.all(d[interior] == 0)
    assert np.any(d[~interior] != 0)
    # 2-D: f = A(y) + B(x) is annihilated away from chunk borders
    A2 = rng.integers(-1000, 1000, size=(50, 1))
    B2 = rng.integers(-1000, 1000, size=(1, 1500))
    d2 = O.lorenzo_field((A2 + B2).astype(np.int32))
    yy, xx = np.meshgrid(np.arange(50), np.arange(1500), indexing="ij")
    assert np.all(d2[(yy % 32 > 0) & (xx % 1024 > 0)] == 0)


def test_lorenzo_small_hand_examples():
    # 2x2 example: q = [[1,2],[3,5]] -> delta = [[1,1],[2,1]]
    assert O.lorenzo_field(np.array([[1, 2], [3, 5]], np.int32)).tolist() == [[1, 1], [2, 1]]
    # 2x2x2: q[z][y][x] = 1 + x + 10 y + 100 z + 1000 xyz
    q = np.zeros((2, 2, 2), np.int32)
    for z in range(2):
        for y in range(2):
            for x in range(2):
                q[z, y, x] = 1 + x + 10 * y + 100 * z + 1000 * x * y * z
    # delta(0,0,0)=1; single differences pick up 1, 10, 100; mixed second
    # differences of a trilinear-free part vanish; the xyz term survives once
    assert O.lorenzo_field(q).tolist() == [[[1, 1], [10, 0]], [[100, 0], [0, 1000]]]
    # 1-D: first differences with a zero ghost in front
    assert O.lorenzo_field(np.array([5, 7, 4], np.int32)).tolist() == [5, 2, -3]


# ------------------------------------------------------------------ code map
def test_code_map_exhaustive():
    lib = O.lib()
    import ctypes
    c = np.zeros(1, np.uint16)
    p = c.ctypes.data_as(ctypes.c_void_p)
    for d in range(-32767, 32768):
        esc = lib.fzo_code_of(d, p)
        code = int(c[0])
        assert esc == 0
        assert code != 0x8000
        assert (code & 0x7FFF) == abs(d)
        assert (code >> 15) == (1 if d < 0 else 0)
        assert lib.fzo_delta_of(code) == d
    for d in [32768, -32768, 2 ** 31 - 1, -(2 ** 31), 100000]:
        code, esc = O.code_of(d)
        assert esc and code == 0x8000


# --------------------------------------------- bitshuffle, flags, sizes, W1
def test_w1_golden():
    g = json.load(open(os.path.join(GOLD, "w1_1d.json")))
    x = np.array(g["x"], np.float32)
    s, st = O.compress(x, g["eb_abs"], O.EB_ABS)
    assert st == 0
    h = stream_np.header(s)
    assert h["ebx2"] == g["ebx2"] and h["inv"] == g["inv"]
    assert O.header_bytes(x.shape) == g["header_bytes"]
    assert len(s) == g["total_bytes"] == h["total"]
    r = stream_np.read(s, x.shape)
    assert r["codes"][0][:5].tolist() == g["codes"]
    assert r["q"].tolist() == g["q"]
    fl = r["flags"][0, 0]
    for b in range(16):
        assert int(fl[b]) == int(g["flags_layer0"].get(str(b), 0))
    assert np.frombuffer(s[656:704].tobytes(), np.uint32).reshape(3, 4).tolist() == g["bricks"]
    y, err = O.decompress(s, x.shape)
    assert err == 0 and y.tolist() == g["x_reconstructed"]
    codes = O.chunk_codes(x, g["inv"], 0)
    assert codes[:5].tolist() == g["codes"] and not codes[5:].any()


@pytest.mark.parametrize("shape,seed", [((33, 70, 130), 21), ((75, 2050), 22), ((100000,), 23), ((5, 3, 2), 24)])
def test_stream_read_independently(shape, seed):
    """An independent numpy reader of the stream recovers rint(x*inv); the
    flags' popcounts equal the header's block count; size identity holds."""
    x = synth.sine_field(shape, seed=seed)
    s, st = O.compress(x, 1e-3, O.EB_REL)
    assert st == 0
    r = stream_np.read(s, shape)
    h = r["header"]
    assert np.array_equal(r["q"], _q_numpy(x, h["inv"]))
    nnz = sum(r["nnz"])
    assert nnz == h["nnz"]
    pop = sum(bin(int(v)).count("1") for v in r["flags"].ravel())
    assert pop == nnz
    units = sum(n + (o + 1) // 2 for n, o in zip(r["nnz"], r["nout"]))
    assert h["total"] == len(s) == r["H"] + 16 * units
    # the chunk table is the exclusive prefix sum of units
    pref = np.concatenate([[0], np.cumsum([n + (o + 1) // 2 for n, o in zip(r["nnz"], r["nout"])])[:-1]])
    assert np.array_equal(r["table"][:, 0], pref)
    # the set bits of all bricks equal the set bits of all codes
    bits_codes = sum(int(np.unpackbits(c.astype('<u2').view(np.uint8)).sum()) for c in r["codes"])
    pl = np.frombuffer(s[r["H"]:].tobytes(), np.uint8)
    assert int(np.unpackbits(pl).sum()) == bits_codes


def test_brick_unit_vector():
    """One nonzero code 1<<j at (step, patch, cell) lands as one brick of plane
    j with exactly the bit 32*(step%4)+cell set (1-D, ABS, inv = 1)."""
    for step, patch, cell, j in [(0, 0, 0, 0), (5, 17, 31, 3), (15, 63, 7, 14)]:
        n = step * 2048 + patch * 32 + cell
        x = np.zeros(32768, np.float32)
        # 1-D delta is a first difference, so a step function of height 2^j
        # starting at n gives exactly one nonzero delta
        x[n:] = 2.0 ** j
        s, st = O.compress(x, 0.5, O.EB_ABS)
        r = stream_np.read(s, x.shape)
        assert r["nnz"] == [1]
        k = step // 4
        assert int(r["flags"][0, k, j]) == 1 << patch
        br = np.frombuffer(s[r["H"]:r["H"] + 16].tobytes(), np.uint32)
        expect = np.zeros(4, np.uint32)
        expect[step % 4] = 1 << cell
        assert br.tolist() == expect.tolist()


def test_all_zero_field_ratio():
    x = np.zeros((64, 64, 64), np.float32)
    s, st = O.compress(x, 1e-3, O.EB_REL)
    assert st == 0 and stream_np.header(s)["nnz"] == 0
    # only header, table and flags: 512 flag bytes per 128 KiB chunk
    assert len(s) == O.header_bytes(x.shape)
    assert x.nbytes / len(s) > 200


# ------------------------------------------------------------ eb parameters
def test_rel_params_against_numpy():
    x = synth.sine_field((20, 30, 40), seed=31)
    p = O.eb_params(x, 1e-3, O.EB_REL)
    lo, hi = float(x.min()), float(x.max())
    assert p["vmin"] == np.float32(lo) and p["vmax"] == np.float32(hi)
    e2 = np.float32(2.0 * (1e-3 * (hi - lo)))
    assert p["ebx2"] == e2 and p["inv"] == np.float32(1.0 / float(e2))
    # constant fields
    p = O.eb_params(np.full(10, 3.0, np.float32), 1e-2, O.EB_REL)
    assert p["ebx2"] == np.float32(2 * 1e-2 * 3.0) and p["status"] == 0
    p = O.eb_params(np.zeros(10, np.float32), 1e-2, O.EB_REL)
    assert p["ebx2"] == np.float32(2e-2) and p["status"] == 0
    # ABS mode records no range
    p = O.eb_params(x, 0.25, O.EB_ABS)
    assert p["ebx2"] == 0.5 and p["inv"] == 2.0 and p["vmin"] == 0 and p["vmax"] == 0


# -------------------------------------------------------------- error paths
def test_error_status_bits():
    x = synth.sine_field((10, 10, 10), seed=1)
    bad = x.copy(); bad[3, 4, 5] = np.nan
    assert O.compress(bad, 1e-3, O.EB_REL)[1] == O.ERR_NONFINITE
    assert O.compress(bad, 1e-3, O.EB_ABS)[1] == O.ERR_NONFINITE
    bad[3, 4, 5] = np.inf
    assert O.compress(bad, 1e-3, O.EB_ABS)[1] == O.ERR_NONFINITE
    big = x * np.float32(1e30)
    assert O.compress(big, 1e-10, O.EB_ABS)[1] == O.ERR_EB_RANGE
    # tiny eb makes ebx2 underflow
    assert O.compress(x, 1e-45, O.EB_ABS)[1] == O.ERR_EB_RANGE


def test_escapes_and_outlier_cap():
    # an offset field at a small eb forces escapes at chunk origins
    x = synth.sine_field((20, 40, 70), seed=2) + np.float32(1000.0)
    s, st = O.compress(x, 1e-3, O.EB_ABS)
    assert st == 0
    h = stream_np.header(s)
    assert h["n_out"] > 0
    r = stream_np.read(s, x.shape)
    assert np.array_equal(r["q"], _q_numpy(x, h["inv"]))
    y, err = O.decompress(s, x.shape)
    assert err == 0
    assert np.array_equal(y, _q_numpy(x, h["inv"]).astype(np.float32) * np.float32(h["ebx2"]))
    # white noise of huge amplitude: almost every delta escapes -> cap
    rng = np.random.default_rng(3)
    w = (rng.standard_normal((16, 32, 64)) * 1e6).astype(np.float32)
    assert O.compress(w, 0.5, O.EB_ABS)[1] == O.ERR_OUTLIER_CAP


def _escapes_per_layer(r, c):
    codes = r["codes"][c]
    return [int(np.count_nonzero(codes[8192 * k:8192 * (k + 1)] == 0x8000)) for k in range(4)]


@pytest.mark.parametrize("shape,count,rows,layer,expect", [
    ((32768,), 150, (0, 8190), 0, 300),        # 1-D: 2 escapes per spike, all in layer 0
    ((32768,), 128, (8192, 16382), 1, 256),    # exactly 256 in one layer
    ((32768,), 129, (8192, 16382), 1, 258),    # just past 256 in one layer
    ((32768,), 512, (16384, 24574), 2, 1024),  # the whole chunk's allowance in one layer
    ((16, 32, 64), 40, (4, 7), 1, 320),        # 3-D: 8 escapes per spike, planes 4-7
    ((32, 1024), 100, (8, 15), 1, 400),        # 2-D: 4 escapes per spike, rows 8-15
])
def test_escapes_concentrated_in_one_layer(shape, count, rows, layer, expect):
    """A chunk may store up to 1024 escaped codes wherever they fall (the
    format caps the chunk, not its layers): a stream whose escapes crowd
    into one layer is valid, reads back to rint(x * inv), and decompresses
    to x (spikes of 100000 on a grid of step 1 are exact)."""
    x = synth.spike_field(shape, count, rows, seed=17)
    s, st = O.compress(x, 0.5, O.EB_ABS)
    assert st == 0
    h = stream_np.header(s)
    assert h["n_out"] == expect
    r = stream_np.read(s, shape)
    per = _escapes_per_layer(r, 0)
    assert per[layer] == expect and sum(per) == expect
    assert np.array_equal(r["q"], x.astype(np.int32))
    y, err = O.decompress(s, shape)
    assert err == 0 and np.array_equal(y, x)


def test_escape_cap_is_per_chunk():
    # 1025 escapes in one chunk: the cap; the same count split over two
    # chunks (1024 + 1) is a valid stream
    x = synth.spike_field((32768,), 512, (16384, 24574), seed=18)
    x[30000:] = np.float32(100000.0)  # one more escape (a step) in layer 3
    assert O.compress(x, 0.5, O.EB_ABS)[1] == O.ERR_OUTLIER_CAP
    x2 = np.concatenate([synth.spike_field((32768,), 512, (16384, 24574), seed=18), np.zeros(32768, np.float32)])
    x2[40000:] = np.float32(100000.0)
    s, st = O.compress(x2, 0.5, O.EB_ABS)
    assert st == 0
    r = stream_np.read(s, x2.shape)
    assert r["nout"] == [1024, 1]
    y, err = O.decompress(s, x2.shape)
    assert err == 0 and np.array_equal(y, x2)


def test_decompress_rejects_bad_streams():
    x = synth.sine_field((10, 20, 30), seed=4)
    s, _ = O.compress(x, 1e-3, O.EB_REL)
    for mutate, code in [(lambda a: a.__setitem__(0, 0), 2), (lambda a: a.__setitem__(4, 9), 3),
                         (lambda a: a.__setitem__(8, 1), 4)]:
        t = s.copy(); mutate(t)
        assert O.decompress(t, x.shape)[1] == code
    assert O.decompress(s[:200], x.shape)[1] == 2
    assert O.decompress(s, (10, 20, 31))[1] == 2


def test_openmp_equals_single_thread():
    x = synth.sine_field((64, 96, 130), seed=5)
    a, _ = O.compress(x, 1e-4, O.EB_REL, threads=1)
    b, _ = O.compress(x, 1e-4, O.EB_REL, threads=8)
    assert np.array_equal(a, b)
    # decompression over chunks in parallel: the same values, the same errors
    ya, ea = O.decompress(a, x.shape)
    yb, eb_ = O.decompress(a, x.shape, threads=8)
    assert ea == eb_ == 0 and np.array_equal(ya.view(np.uint32), yb.view(np.uint32))
    for shape, seed, glob in (((70, 2100), 6, False), ((100001,), 7, False), ((40, 70, 130), 8, True)):
        xs = synth.sine_field(shape, seed=seed) + np.float32(300.0)  # escapes at chunk origins
        s, st = O.compress(xs, 1e-3, O.EB_ABS, global_lorenzo=glob)
        assert st == 0
        y1, e1 = O.decompress(s, shape)
        y8, e8 = O.decompress(s, shape, threads=8)
        assert e1 == e8 == 0 and np.array_equal(y1.view(np.uint32), y8.view(np.uint32))
    bad = a.copy()
    bad[128 + 8 * 3] ^= 1  # a chunk offset off by one unit
    assert O.decompress(bad, x.shape)[1] == O.decompress(bad, x.shape, threads=8)[1] == 2
