"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/fz.h declares, sizes agree with the oracle's format
arithmetic, argument errors return immediately, and the header parser reads
an oracle-made stream."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fz_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 6
    L = fz.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fz.SYMBOLS)


@pytest.mark.parametrize("shape", [(64, 64, 64), (100, 500, 500), (1800, 3600), (7,), (1, 1, 1), (33, 1, 1025),
                                   (512, 512, 512), (280953867,)])
def test_sizes_match_oracle(shape):
    assert fz.header_bytes(shape) == O.header_bytes(shape)
    assert fz.compress_bound(shape) >= O.bound(shape)


# a 256-byte aligned stand-in pointer: every call below fails an argument
# check before anything is enqueued, so it is never dereferenced
P = ctypes.c_void_p(4096)


def test_argument_errors_return_immediately():
    L = fz.lib()
    d = fz.dims_of((10, 10))
    assert L.fz_compress(None, ctypes.byref(d), 1e-3, 1, P, None) == 1
    assert L.fz_compress(P, ctypes.byref(d), -1.0, 1, P, None) == 1
    assert L.fz_compress(P, ctypes.byref(d), float("nan"), 1, P, None) == 1
    assert L.fz_compress(P, ctypes.byref(d), 1e-3, 7, P, None) == 1
    assert L.fz_compress(P, ctypes.byref(d), 1e-45, 0, P, None) == 4
    # point-wise relative mode: a step S = floor(eps 2^24 / (1 + eps)) below 2 is out of range
    assert L.fz_compress(P, ctypes.byref(d), 1e-8, 2, P, None) == 4
    assert L.fz_compress(P, ctypes.byref(d), 1.1e-7, 2, P, None) == 4
    assert L.fz_compress(P, ctypes.byref(d), 1e-3, 3, P, None) == 1
    # fp64 input: grid modes only; 2 eb below the smallest normal double is out of range
    assert L.fz_compress_f64(P, ctypes.byref(d), 1e-3, 2, P, None) == 1
    assert L.fz_compress_f64(None, ctypes.byref(d), 1e-3, 0, P, None) == 1
    assert L.fz_compress_f64(P, ctypes.byref(d), float("inf"), 0, P, None) == 1
    assert L.fz_compress_f64(P, ctypes.byref(d), 1e-310, 0, P, None) == 4
    assert L.fz_decompress_f64(None, 1 << 20, P, ctypes.byref(d), None, None) == 1
    # field-global predictor: the chunk-local checks, and a work buffer is required
    assert L.fz_compress_global(P, ctypes.byref(d), -1.0, 1, P, None) == 1
    assert L.fz_compress_global(P, ctypes.byref(d), 1e-8, 2, P, None) == 4
    assert L.fz_decompress_global(P, 1 << 20, P, ctypes.byref(d), None, None, None) == 1
    bad = fz.FzDims()
    bad.rank = 4
    assert L.fz_compress(P, ctypes.byref(bad), 1e-3, 1, P, None) == 1
    bad.rank = 2
    bad.n[0], bad.n[1] = 0, 5
    assert L.fz_compress_bound(ctypes.byref(bad)) == 0
    assert L.fz_decompress(None, 1 << 20, P, ctypes.byref(d), None, None) == 1
    assert fz.lib().fz_strerror(6) == b"malformed stream"


def test_misaligned_and_short_buffers_are_argument_errors():
    """Buffers the kernels address with atomics and 8/16-byte accesses must
    be aligned (256 bytes for whole buffers, 4 for the error word, 8 for the
    quality report), and a decompression's stream_bytes must cover at least
    the header, table and flags: otherwise FZ_ERR_ARG before any launch."""
    L = fz.lib()
    d = fz.dims_of((10, 10))
    hb = fz.header_bytes((10, 10))
    off = ctypes.c_void_p(4096 + 16)
    for fn in (L.fz_compress, L.fz_compress_global, L.fz_compress_f64):
        assert fn(P, ctypes.byref(d), 1e-3, 1, off, None) == 1  # output not on 256 bytes
    assert L.fz_compress(ctypes.c_void_p(4098), ctypes.byref(d), 1e-3, 1, P, None) == 1  # input not on 4
    assert L.fz_compress_f64(ctypes.c_void_p(4100), ctypes.byref(d), 1e-3, 1, P, None) == 1  # fp64 input not on 8
    for fn in (L.fz_decompress, L.fz_decompress_f64):
        assert fn(off, 1 << 20, P, ctypes.byref(d), None, None) == 1          # stream not on 256
        assert fn(P, 1 << 20, P, ctypes.byref(d), ctypes.c_void_p(4098), None) == 1  # error word not on 4
        assert fn(P, hb - 1, P, ctypes.byref(d), None, None) == 1             # stream shorter than its header
    assert L.fz_decompress(P, 1 << 20, ctypes.c_void_p(4098), ctypes.byref(d), None, None) == 1
    assert L.fz_decompress_f64(P, 1 << 20, ctypes.c_void_p(4100), ctypes.byref(d), None, None) == 1
    assert L.fz_decompress_global(P, 1 << 20, P, ctypes.byref(d), None, off, None) == 1  # work not on 256
    assert L.fz_decompress_global(P, hb - 1, P, ctypes.byref(d), None, P, None) == 1
    assert L.fz_quality(P, P, ctypes.byref(d), ctypes.c_void_p(4100), P, None) == 1  # report not on 8
    assert L.fz_quality(P, P, ctypes.byref(d), P, off, None) == 1                    # work not on 256
    # batch jobs and server requests make the same checks
    jobs = (fz.FzCompressJob * 1)()
    jobs[0].d_in, jobs[0].d_out, jobs[0].eb, jobs[0].eb_mode = 4096, 4096 + 16, 1e-3, fz.FZ_EB_REL
    jobs[0].dims = d
    h = ctypes.c_void_p(123)
    assert L.fz_batch_create_compress(1, jobs, ctypes.byref(h)) == 1 and not h.value
    djobs = (fz.FzDecompressJob * 1)()
    djobs[0].d_stream, djobs[0].d_out, djobs[0].dims, djobs[0].stream_bytes = 4096, 4096, d, hb - 1
    assert L.fz_batch_create_decompress(1, djobs, ctypes.byref(h)) == 1
    djobs[0].stream_bytes, djobs[0].d_stream = 1 << 20, 4096 + 64
    assert L.fz_batch_create_decompress(1, djobs, ctypes.byref(h)) == 1
    # the binding refuses the same before calling in
    import torch
    with pytest.raises(ValueError):
        fz._check_buffer(torch.zeros(4), "t", (torch.float32,), 4)  # a host tensor


def test_stream_info_parses_oracle_header():
    x = synth.sine_field((20, 40, 70), seed=9)
    s, st = O.compress(x, 1e-3, O.EB_REL)
    info = fz.stream_info(s[:128].tobytes())
    assert info["total_bytes"] == len(s)
    assert info["rank"] == 3 and info["n"] == [20, 40, 70]
    assert info["header_bytes"] == O.header_bytes(x.shape)
    assert info["status"] == st == 0
    with pytest.raises(fz.FzError):
        fz.stream_info(b"\0" * 128)


def test_size_limits():
    """The library's documented limits: extents up to 2^40, a contiguous
    extent below 2^25 for rank 2 and 3, fewer than 2^31 chunks."""
    L = fz.lib()

    def bound(rank, n):
        d = fz.FzDims()
        d.rank = rank
        for i in range(3):
            d.n[i] = n[i] if i < len(n) else 1
        return L.fz_compress_bound(ctypes.byref(d)), d

    assert bound(2, (4, (1 << 25) - 1))[0] > 0
    b, d = bound(2, (4, 1 << 25))
    assert b == 0
    assert L.fz_compress(P, ctypes.byref(d), 1e-3, 1, P, None) == 1
    assert bound(3, (2, 3, 1 << 25))[0] == 0
    assert bound(1, (1 << 40,))[0] > 0
    assert bound(1, ((1 << 40) + 1,))[0] == 0
    # 2^31 chunks: 2^16 x 2^15 chunk boxes of 32 x 1024
    assert bound(2, (32 << 16, (1 << 15) * 1024 - 1))[0] == 0  # contiguous extent too large first
    assert bound(3, (16 << 11, 32 << 10, 64 << 10))[0] == 0     # 2^31 chunks
    assert bound(3, (16 << 11, 32 << 10, (64 << 10) - 64))[0] > 0


def test_batch_create_rejects_bad_jobs():
    """Invalid jobs are refused before anything touches a device."""
    L = fz.lib()
    jobs = (fz.FzCompressJob * 2)()
    for j in jobs:
        j.d_in, j.d_out, j.eb, j.eb_mode = 4096, 4096, 1e-3, fz.FZ_EB_REL
        j.dims = fz.dims_of((10, 10))
    jobs[1].eb = -1.0
    h = ctypes.c_void_p(123)
    assert L.fz_batch_create_compress(2, jobs, ctypes.byref(h)) == 1
    assert not h.value
    jobs[1].eb, jobs[1].eb_mode = 1e-45, fz.FZ_EB_ABS
    assert L.fz_batch_create_compress(2, jobs, ctypes.byref(h)) == 4
    assert L.fz_batch_create_compress(0, jobs, ctypes.byref(h)) == 1
    djobs = (fz.FzDecompressJob * 1)()
    djobs[0].d_stream, djobs[0].d_out, djobs[0].dims = None, 4096, fz.dims_of((5,))
    assert L.fz_batch_create_decompress(1, djobs, ctypes.byref(h)) == 1
    assert L.fz_batch_run(None, None) == 1
    assert L.fz_batch_destroy(None) == 1


def test_server_argument_errors():
    """Server calls refuse bad arguments without touching a device."""
    L = fz.lib()
    h = ctypes.c_void_p(7)
    assert L.fz_server_create(0, 2, 8, ctypes.byref(h)) == 1 and not h.value
    assert L.fz_server_create(1 << 30, 0, 8, ctypes.byref(h)) == 1
    assert L.fz_server_create(1 << 30, 2, 0, ctypes.byref(h)) == 1
    t = ctypes.c_uint64()
    r = fz.FzRequest(kind=0, eb_mode=1, eb=1e-3, dims=fz.dims_of((10,)), d_in=4096, d_out=4096, d_err=None,
                     hbm_bytes=0, stream_bytes=0, ready_event=None)
    assert L.fz_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == 1
    assert L.fz_server_wait(None, 1, None) == 1
    assert L.fz_server_destroy(None) == 1


def test_quality_argument_errors():
    L = fz.lib()
    d = fz.dims_of((1000, 3))
    p = ctypes.c_void_p(256)
    work = L.fz_quality_work_bytes(ctypes.byref(d))
    assert 32 <= work <= 64 * 1024 and work % 32 == 0
    assert L.fz_quality_work_bytes(ctypes.byref(fz.dims_of((512, 512, 512)))) == 2048 * 32
    assert L.fz_quality(None, p, ctypes.byref(d), p, p, None) == 1
    assert L.fz_quality(p, None, ctypes.byref(d), p, p, None) == 1
    assert L.fz_quality(p, p, ctypes.byref(d), None, p, None) == 1
    assert L.fz_quality(p, p, ctypes.byref(d), p, None, None) == 1
    assert L.fz_quality(p, p, None, p, p, None) == 1
    bad = fz.FzDims()
    bad.rank = 2
    bad.n[0], bad.n[1] = 4, 0
    assert L.fz_quality_work_bytes(ctypes.byref(bad)) == 0
    assert L.fz_quality(p, p, ctypes.byref(bad), p, p, None) == 1
    assert ctypes.sizeof(fz.FzQuality) == 56


def test_ablation_argument_errors():
    L = fz.lib()
    p = ctypes.c_void_p(256)
    good = fz.dims_of((32, 64, 128))
    for shape in [(32, 64), (32, 64, 100), (20, 64, 128), (32, 48, 128)]:
        d = fz.dims_of(shape)
        assert L.fz_abl_pred_quant(2, p, ctypes.byref(d), 100.0, p, p, None) == 1, shape
        assert L.fz_abl_bitshuffle(p, ctypes.byref(d), p, None) == 1, shape
        assert L.fz_abl_mark(p, ctypes.byref(d), p, None) == 1, shape
        assert L.fz_abl_bitshuffle_mark(p, ctypes.byref(d), p, p, None) == 1, shape
        assert L.fz_abl_bitshuffle_ballot(p, ctypes.byref(d), p, None) == 1, shape
        assert L.fz_abl_bitshuffle_mark_ballot(p, ctypes.byref(d), p, p, None) == 1, shape
        assert L.fz_abl_encode(p, p, ctypes.byref(d), p, p, None) == 1, shape
    assert L.fz_abl_pred_quant(3, p, ctypes.byref(good), 100.0, p, p, None) == 1
    assert L.fz_abl_pred_quant(1, p, ctypes.byref(good), 100.0, p, None, None) == 1
    assert L.fz_abl_pred_quant(2, p, ctypes.byref(good), float("inf"), p, None, None) == 1
    assert L.fz_abl_pred_quant(2, p, ctypes.byref(good), 0.0, p, None, None) == 1
    assert L.fz_abl_pred_quant(2, None, ctypes.byref(good), 100.0, p, None, None) == 1
    assert L.fz_abl_encode(p, p, ctypes.byref(good), None, p, None) == 1


@pytest.mark.parametrize("shape", [(1,), (70001,), (45, 1030), (20, 40, 70), (512, 512, 512)])
def test_f64_bound(shape):
    """The fp64 output buffer holds the fp32 one plus the integers q and the
    range pass's partials."""
    n = int(np.prod(shape))
    b32, b64 = fz.compress_bound(shape), fz.compress_bound(shape, f64=True)
    assert b64 >= b32 + 4 * n and b64 % 4 == 0


@pytest.mark.parametrize("shape", [(1,), (70001,), (45, 1030), (20, 40, 70), (512, 512, 512)])
def test_global_sizes(shape):
    """The field-global predictor's output buffer holds the fp32 one plus the
    integers; its decompression work holds one u32 per chunk-box segment of
    every line along every axis."""
    n = int(np.prod(shape))
    assert fz.compress_bound(shape, global_lorenzo=True) >= fz.compress_bound(shape) + 4 * n
    box = {1: (32768,), 2: (32, 1024), 3: (16, 32, 64)}[len(shape)]
    total = sum(4 * (n // shape[a]) * -(-shape[a] // box[a]) for a in range(len(shape)))
    assert fz.lib().fz_decompress_global_work_bytes(ctypes.byref(fz.dims_of(shape))) == total

@pytest.mark.parametrize("shape", [(512, 512, 512), (100, 500, 500), (1800, 3600), (64, 64, 64), (7,), (1 << 27,)])
def test_bound_is_stream_plus_scratch(shape):
    """fz_compress_bound = the worst-case stream, then the scratch with one
    staging slot per persistent workgroup (at most 768): below 0.7 times the
    input for the large fields; fz_stream_bound is the stream part alone."""
    n = int(np.prod(shape))
    b, sb = fz.compress_bound(shape), fz.stream_bound(shape)
    assert 0 < sb < b
    assert sb == O.bound(shape)  # the oracle's own worst-case stream size
    slot = 16 * 4 * 64 * 16 + 1024 * 8
    chunks = -(-n // 32768) if len(shape) == 1 else None
    if n * 4 >= 100 << 20:
        assert b <= 0.7 * 4 * n, (b, 4 * n)
    if chunks is not None:
        assert b - sb >= min(chunks, 768) * slot


def test_noalloc_argument_checks_on_the_host():
    """fz_compress_noalloc rejects, before touching any device, a missing
    pointer, an output smaller than the stream bound and a field whose
    scratch does not fit the library's array (FZ_ERR_ARG = 1)."""
    L = fz.lib()
    p = ctypes.c_void_p(256)  # never dereferenced: every call below fails its checks first
    d = fz.dims_of((64, 64, 64))
    sb = fz.stream_bound((64, 64, 64))
    assert L.fz_compress_noalloc(None, ctypes.byref(d), 1e-3, 1, p, sb, None) == 1
    assert L.fz_compress_noalloc(p, ctypes.byref(d), 1e-3, 1, None, sb, None) == 1
    assert L.fz_compress_noalloc(p, ctypes.byref(d), 1e-3, 1, p, sb - 1, None) == 1
    big = fz.dims_of((1 << 36,))  # 2^21 chunks
    assert L.fz_compress_noalloc(p, ctypes.byref(big), 1e-3, 1, p, 1 << 62, None) == 1

