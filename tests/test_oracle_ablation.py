"""Pins of the ablation-pipeline oracle (CPU only): the two code mappings at
their boundaries, the tile layout on single-bit inputs, the step and patch
order against the C oracle's code order, flags and encoding on constructed
tiles, and the round trip of codes through tiles."""
import numpy as np
import pytest

from oracle import ablation as A
from oracle import oracle as O
import synth


def field(seed=1, shape=(32, 64, 128)):
    return synth.sine_field(shape, seed=seed)


def test_code_mappings_at_their_boundaries():
    # a field whose only nonzero chunk-local delta sits at its first cell: d = q(0,0,0)
    for q0, v1, out1, v2 in [(0, 512, 0, 0), (511, 1023, 0, 511), (-511, 1, 0, 0x8000 | 511), (512, 0, 512, 512),
                             (-512, 0, -512, 0x8000 | 512), (32767, 0, 32767, 32767), (32768, 0, 32768, 0x8000),
                             (-40000, 0, -40000, 0x8000)]:
        x = np.zeros((16, 32, 64), np.float32)
        x[0, 0, 0] = np.float32(q0)
        c1, o1 = A.pred_quant_v1(x, 1.0)
        c2 = A.pred_quant_v2(x, 1.0)
        assert c1.reshape(-1)[0] == v1 and o1.reshape(-1)[0] == out1, q0
        assert c2.reshape(-1)[0] == v2, q0
        # the neighbours along x, y and z see -q0 (the Lorenzo stencil), the rest 0
        assert c2.reshape(x.shape)[0, 0, 2] == 0 and c1.reshape(x.shape)[0, 0, 2] == 512


def test_v2_codes_match_the_oracle_code_mapping():
    x = field()
    inv = np.float32(1.0 / 0.01)
    c2 = A.pred_quant_v2(x, inv).reshape(-1)
    d = A.deltas(x, inv).reshape(-1)
    for i in np.random.default_rng(0).choice(c2.size, 300, replace=False):
        assert c2[i] == O.code_of(int(d[i]))[0]


def test_step_and_patch_order_match_the_format_code_order():
    x = field(seed=2)
    inv = np.float32(1.0 / 0.004)
    c2 = A.pred_quant_v2(x, inv).reshape(x.shape)
    planes = A.steps_of(c2)
    for c in range(4):  # the C oracle's codes of chunk c: step * 2048 + patch * 32 + cell
        ref = O.chunk_codes(x, inv, c).reshape(16, 64, 32)
        cells = planes[16 * c:16 * (c + 1)].reshape(16, 8, 4, 8, 8).transpose(0, 3, 1, 2, 4).reshape(16, 64, 32)
        assert np.array_equal(cells, ref), c


def test_tile_layout_on_single_bits():
    codes = np.zeros((16, 32, 64), np.uint16)
    # patch p = 3 + 8 * 5 covers rows 12..15, columns 40..47; cell m = 8 * 2 + 6 is row 14, column 46
    codes[7, 14, 46] = 1 << 9
    t = A.bitshuffle(codes)
    assert t.shape == (16, 1024)
    nz = np.argwhere(t != 0)
    assert nz.tolist() == [[7, 9 * 64 + 43]]
    assert t[7, 9 * 64 + 43] == 1 << 22


def test_bitshuffle_round_trip():
    rng = np.random.default_rng(3)
    codes = rng.integers(0, 1 << 16, size=(16, 64, 128), dtype=np.uint16)
    t = A.bitshuffle(codes).reshape(-1, 16, 64)
    back = np.zeros((t.shape[0], 64, 32), np.uint32)
    for b in range(16):
        back |= ((t[:, b, :, None] >> np.arange(32, dtype=np.uint32)) & 1) << b
    planes = A.steps_of(codes).reshape(-1, 8, 4, 8, 8).transpose(0, 3, 1, 2, 4).reshape(-1, 64, 32)
    assert np.array_equal(back, planes)


def test_mark_and_encode_on_constructed_tiles():
    tiles = np.zeros((3, 1024), np.uint32)
    tiles[0, 4 * 5 + 2] = 7        # step 0, block 5
    tiles[0, 4 * 200] = 1          # step 0, block 200
    tiles[2, 4 * 63 + 3] = 0xFFFF  # step 2, block 63
    f = A.mark(tiles)
    assert f.shape == (3, 4)
    assert f[0].tolist() == [1 << 5, 0, 0, 1 << (200 - 192)]
    assert f[1].tolist() == [0, 0, 0, 0]
    assert f[2].tolist() == [1 << 63, 0, 0, 0]
    off, pay = A.encode(tiles, f)
    assert off.tolist() == [0, 2, 2, 3]
    blocks = pay.view(np.uint32).reshape(-1, 4)
    assert blocks.tolist() == [[0, 0, 7, 0], [1, 0, 0, 0], [0, 0, 0, 0xFFFF]]


def test_v1_shift_fills_blocks_that_v2_leaves_zero():
    # the effect the encoder ablation measures: zero deltas give code r in v1
    x = np.zeros((16, 32, 64), np.float32)
    c1, _ = A.pred_quant_v1(x, 1.0)
    c2 = A.pred_quant_v2(x, 1.0)
    f1 = A.mark(A.bitshuffle(c1.reshape(x.shape)))
    f2 = A.mark(A.bitshuffle(c2.reshape(x.shape)))
    assert int(sum(bin(int(w)).count("1") for w in f2.reshape(-1))) == 0
    assert int(sum(bin(int(w)).count("1") for w in f1.reshape(-1))) == 16 * 16  # plane 9 (512) in every block group
