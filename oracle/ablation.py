"""ORACLE of the per-kernel ablation pipeline -- test infrastructure only.

Only the tests may import this module; the product library never does.
Plain numpy, written from the definitions (the stages the paper compares in
Sec. 4.5), on 3-D fields whose extents are multiples of the 16 x 32 x 64
chunk box.  q and the chunk-local Lorenzo differences come from the C oracle
(``oracle.prequant``, ``oracle.lorenzo_field``), which its own pins cover.

* pred-quant v1, the original dual-quantization (Sec. 2.3): the code is
  d + r for -r < d < r (r = 512), else 0 with d kept in a dense outlier array.
* pred-quant v2, the optimized one (Sec. 3.2): the 16-bit sign-magnitude code
  of d, 0x8000 when |d| > 32767.
* bitshuffle (Sec. 3.3): per step (one z-plane of a chunk) a tile of 1024 u32
  words; word b * 64 + p holds bit b of the 32 codes of patch p (bit m = cell
  m; cell m is row m // 8, column m % 8 of the patch; patch p covers rows
  4 * (p % 8) .., columns 8 * (p // 8) ..).
* mark (Sec. 3.4): block beta = words 4 beta .. 4 beta + 3 (plane beta // 16 of
  128 consecutive codes); bit beta % 64 of flag word beta // 64 is set when the
  block is nonzero.
* encode (Sec. 3.4): the exclusive prefix sum of the per-step nonzero-block
  counts, and the nonzero blocks in order.
Steps are numbered chunk by chunk (chunks in row-major order), z-planes in order.
"""
import numpy as np

from oracle import oracle as O

RADIUS = 512
BOX = (16, 32, 64)


def deltas(x, inv):
    """Chunk-local Lorenzo differences of q = rint(x * inv), row-major int32."""
    q, st = O.prequant(np.ascontiguousarray(x, np.float32), np.float32(inv))
    if st:
        raise ValueError("prequantization status %d (non-finite or |x * inv| >= 2^31)" % st)
    return O.lorenzo_field(q.reshape(x.shape))


def pred_quant_v1(x, inv):
    d = deltas(x, inv).astype(np.int64)
    inside = (d > -RADIUS) & (d < RADIUS)
    codes = np.where(inside, d + RADIUS, 0).astype(np.uint16)
    outliers = np.where(inside, 0, d).astype(np.int32)
    return codes, outliers


def pred_quant_v2(x, inv):
    d = deltas(x, inv).astype(np.int64)
    mag = np.abs(d)
    codes = np.where(mag <= 32767, np.where(d < 0, 0x8000, 0) | mag, 0x8000)
    return codes.astype(np.uint16)


def steps_of(codes3d):
    """The codes as (steps, 32, 64) planes in step order."""
    nz, ny, nx = codes3d.shape
    gz, gy, gx = nz // BOX[0], ny // BOX[1], nx // BOX[2]
    c = codes3d.reshape(gz, BOX[0], gy, BOX[1], gx, BOX[2])
    c = c.transpose(0, 2, 4, 1, 3, 5)  # chunk (z, y, x), plane z, row, column
    return c.reshape(gz * gy * gx * BOX[0], BOX[1], BOX[2])


def bitshuffle(codes3d):
    """Tiles (steps, 1024) u32 of row-major codes of the field's shape."""
    planes = steps_of(np.asarray(codes3d, np.uint16)).astype(np.uint32)
    s = planes.shape[0]
    # (step, py, r, px, c) -> patch p = py + 8 px, cell m = 8 r + c
    cells = planes.reshape(s, 8, 4, 8, 8).transpose(0, 3, 1, 2, 4).reshape(s, 64, 32)
    tiles = np.zeros((s, 16, 64), np.uint32)
    for b in range(16):
        bits = (cells >> b) & 1
        tiles[:, b, :] = (bits << np.arange(32, dtype=np.uint32)).sum(axis=2, dtype=np.uint64).astype(np.uint32)
    return tiles.reshape(s, 1024)


def mark(tiles):
    """Flags (steps, 4) u64."""
    nzb = (tiles.reshape(tiles.shape[0], 256, 4) != 0).any(axis=2)
    weights = np.uint64(1) << np.arange(64, dtype=np.uint64)
    return (nzb.reshape(-1, 4, 64).astype(np.uint64) * weights).sum(axis=2, dtype=np.uint64)


def encode(tiles, flags):
    """Exclusive offsets (steps + 1, in 16-byte blocks) and the payload bytes."""
    blocks = tiles.reshape(tiles.shape[0], 256, 4)
    nzb = np.zeros((tiles.shape[0], 256), bool)
    for w in range(4):
        nzb[:, 64 * w:64 * (w + 1)] = ((flags[:, w:w + 1] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)) != 0
    counts = nzb.sum(axis=1).astype(np.uint64)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint64)
    payload = blocks[nzb].astype(np.uint32).tobytes()
    return offsets, np.frombuffer(payload, np.uint8)
