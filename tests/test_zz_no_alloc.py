"""fz_compress_noalloc (the compression entry point that allocates nothing,
its scratch in the library's own device array) against fz_compress, through
the C ABI: the same stream byte for byte on two calls in a row, the second
on a smaller field (the array keeps the first call's contents, so whatever
must start at zero has to be cleared by the call itself), in both bound
modes, with an output buffer of only the stream bound.  The streams are also
decompressed and compared with the oracle's reconstruction of its own
stream."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu

CASES = [
    # (shape, generator, eb, mode): the second of each pair is smaller
    [((96, 200, 333), "sine", 1e-3, "rel"), ((40, 70, 130), "sine", 1e-3, "rel")],
    [((700, 1500), "sine", 1e-4, "rel"), ((64, 64), "sine", 1e-2, "abs")],
    [((128, 128, 128), "offset", 1e-3, "rel"), ((7, 9, 1031), "offset", 1e-3, "rel")],
]


def field(shape, kind, seed):
    x = synth.sine_field(shape, seed=seed)
    if kind == "offset":  # escapes in every chunk
        x = (x + np.float32(1000.0)).astype(np.float32)
    return x


def stream_of(buf):
    return buf[:fz.stream_size(buf)].cpu().numpy()


@pytest.mark.parametrize("pair", range(len(CASES)))
def test_noalloc_matches_fz_compress(pair):
    torch.cuda.synchronize()
    for k, (shape, kind, eb, mode) in enumerate(CASES[pair]):
        print("no-alloc case", pair, k, shape, kind, eb, mode, flush=True)
        x = field(shape, kind, seed=50 + 10 * pair + k)
        xt = torch.from_numpy(x).cuda()
        dims = fz.dims_of(shape)
        need = int(fz.lib().fz_stream_bound(ctypes.byref(dims)))
        out = torch.empty(need, dtype=torch.uint8, device="cuda")
        rc = fz.lib().fz_compress_noalloc(ctypes.c_void_p(xt.data_ptr()), ctypes.byref(dims), float(eb),
                                          fz._mode(mode), ctypes.c_void_p(out.data_ptr()), need,
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        ref = fz.compress(xt, eb, mode)
        torch.cuda.synchronize()
        a, b = stream_of(out), stream_of(ref)
        assert fz.stream_info(out)["status"] == 0
        assert a.size == b.size and np.array_equal(a, b), (pair, k)
        y = fz.decompress(out, shape)
        torch.cuda.synchronize()
        ys, st = O.compress(x, eb, O.EB_REL if mode == "rel" else O.EB_ABS)
        assert st == 0 and np.array_equal(a, ys)
        yo, err = O.decompress(ys, shape)
        assert err == 0 and np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32))


def test_noalloc_rejects_short_output_and_oversized_fields():
    x = torch.from_numpy(synth.sine_field((16, 32, 64), seed=3)).cuda()
    dims = fz.dims_of(x.shape)
    need = int(fz.lib().fz_stream_bound(ctypes.byref(dims)))
    out = torch.empty(need, dtype=torch.uint8, device="cuda")
    L = fz.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.fz_compress_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.byref(dims), 1e-3, 1,
                                 ctypes.c_void_p(out.data_ptr()), need - 1, s) == 1
    big = fz.dims_of((1 << 36,))  # 2^21 chunks: its scratch does not fit the array
    assert L.fz_compress_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.byref(big), 1e-3, 1,
                                 ctypes.c_void_p(out.data_ptr()), 1 << 62, s) == 1
    torch.cuda.synchronize()
