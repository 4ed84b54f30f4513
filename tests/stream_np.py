"""Independent numpy reader of the v1 stream, used to pin the oracle.

Written from the stream-format definition without reusing any oracle code: it
parses the header, chunk table, flags and bricks with numpy bit operations,
rebuilds every chunk's codes, decodes them, and undoes the chunk-local Lorenzo
predictor with numpy cumulative sums.  Tests compare what it reads back with
quantities the paper fixes independently of the format (the prequantized
integers of Sec. 2.3).
"""
import numpy as np

HEADER = 128
BOX = {3: (16, 32, 64), 2: (32, 1024), 1: (32768,)}
ROWS_PER_LAYER = {3: 4, 2: 8, 1: 8192}


def header(s):
    s = np.asarray(s, dtype=np.uint8)
    h = s[:HEADER].tobytes()
    u32 = lambda o: int.from_bytes(h[o:o + 4], "little")
    u64 = lambda o: int.from_bytes(h[o:o + 8], "little")
    u16 = lambda o: int.from_bytes(h[o:o + 2], "little")
    return dict(
        magic=u32(0), version=u16(4), header_bytes=u16(6), status=u32(8), dtype=h[12], rank=h[13],
        eb_mode=h[14], dims=[u64(16), u64(24), u64(32)],
        eb=np.frombuffer(h[40:48], np.float64)[0], ebx2=np.frombuffer(h[48:52], np.float32)[0],
        inv=np.frombuffer(h[52:56], np.float32)[0], vmin=np.frombuffer(h[56:60], np.float32)[0],
        vmax=np.frombuffer(h[60:64], np.float32)[0], chunk=[u16(64), u16(66), u16(68)], n_chunks=u32(72),
        nnz=u64(80), n_out=u64(88), total=u64(96))


def cell_coords(rank):
    """(s, p, m) -> box-relative coordinates for all 32768 code indices."""
    n = np.arange(32768)
    s, p, m = n // 2048, (n // 32) % 64, n % 32
    if rank == 3:
        return (s, 4 * (p % 8) + m // 8, 8 * (p // 8) + m % 8)
    if rank == 2:
        return (2 * s + m // 16, 16 * p + m % 16)
    return (2048 * s + 32 * p + m,)


def read(s, shape):
    """Return dict with per-chunk codes, deltas and the reconstructed q field."""
    s = np.asarray(s, dtype=np.uint8)
    h = header(s)
    rank = len(shape)
    box = BOX[rank]
    grid = [-(-shape[i] // box[i]) for i in range(rank)]
    nch = int(np.prod(grid))
    assert h["n_chunks"] == nch
    table = s[HEADER:HEADER + 8 * nch].view(np.uint32).reshape(nch, 2)
    tab_bytes = -(-8 * nch // 16) * 16
    flags = s[HEADER + tab_bytes:HEADER + tab_bytes + 512 * nch].view(np.uint64).reshape(nch, 4, 16)
    H = HEADER + tab_bytes + 512 * nch
    payload = s[H:h["total"]]
    coords = cell_coords(rank)
    q = np.zeros(shape, dtype=np.uint32)
    codes_all, nnz_all, nout_all = [], [], []
    for c in range(nch):
        ci = np.unravel_index(c, grid)
        org = [ci[i] * box[i] for i in range(rank)]
        ext = [min(box[i], shape[i] - org[i]) for i in range(rank)]
        off, nout = int(table[c, 0]), int(table[c, 1])
        # bits of every brick present, in (layer, plane, patch) order
        bits = np.zeros((4, 16, 64), dtype=bool)
        for k in range(4):
            for b in range(16):
                f = int(flags[c, k, b])
                bits[k, b] = [(f >> p) & 1 for p in range(64)]
        nnz = int(bits.sum())
        bricks = payload[16 * off:16 * (off + nnz)].view(np.uint32).reshape(nnz, 4)
        codes = np.zeros(32768, dtype=np.uint32)
        kk, bb, pp = np.nonzero(bits)  # row-major order == stream order
        for i in range(nnz):
            k, b, p = kk[i], bb[i], pp[i]
            for t in range(4):
                w = int(bricks[i, t])
                m = np.arange(32)
                sel = ((w >> m) & 1).astype(bool)
                idx = (4 * k + t) * 2048 + 32 * p + m[sel]
                codes[idx] |= np.uint32(1 << b)
        pairs = payload[16 * (off + nnz):16 * (off + nnz) + 8 * nout].view(np.uint32).reshape(nout, 2)
        mag = (codes & 0x7FFF).astype(np.int64)
        delta = np.where(codes & 0x8000, -mag, mag)
        esc = np.nonzero(codes == 0x8000)[0]
        assert len(esc) == nout and np.array_equal(esc, pairs[:, 0])
        delta[esc] = pairs[:, 1].view(np.int32)
        # scatter into the clipped box and undo Lorenzo with cumulative sums
        inside = np.ones(32768, dtype=bool)
        for i in range(rank):
            inside &= coords[i] < ext[i]
        B = np.zeros(ext, dtype=np.uint32)
        B[tuple(cc[inside] for cc in coords)] = delta[inside].astype(np.int64).astype(np.uint32)
        for ax in reversed(range(rank)):
            B = np.cumsum(B, axis=ax, dtype=np.uint32)
        q[tuple(slice(org[i], org[i] + ext[i]) for i in range(rank))] = B
        codes_all.append(codes)
        nnz_all.append(nnz)
        nout_all.append(nout)
    return dict(header=h, q=q.view(np.int32), codes=codes_all, nnz=nnz_all, nout=nout_all, flags=flags,
                table=table, H=H)
