"""A seeded sweep of the GPU path against the oracle through the C ABI.

Each case draws a rank, extents (often a chunk box plus or minus one, and
contiguous extents that are not multiples of 4), a value recipe, an error-bound
mode and a bound, all from a fixed seed.  The recipes include smooth modes,
heavy-tailed lognormal values, white noise (escapes, and at small bounds the
escape cap), blocks of exact zeros, signed zeros, constant patches and fp32
denormals.  The bar is that of the parity tests: the same status as the
oracle, and when it is 0, the same stream bytes and the same reconstruction
bits.
"""
import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu

BOX = {1: (32768,), 2: (32, 1024), 3: (16, 32, 64)}
MAX_VALUES = 400_000


def draw_shape(rng, rank):
    while True:
        shape = []
        for b in BOX[rank]:
            k = int(rng.integers(0, 4))
            base = b * int(rng.integers(1, 3)) if rank > 1 else b * int(rng.integers(1, 4))
            ext = {0: base, 1: base + 1, 2: max(1, base - 1), 3: int(rng.integers(1, 2 * b + 1))}[k]
            shape.append(ext)
        shape = tuple(shape)
        if np.prod(shape) <= MAX_VALUES:
            return shape


def draw_field(rng, shape, seed):
    kind = ["sine", "lognormal", "noise", "zeros_block", "signed_zero", "denormal", "patches"][int(rng.integers(0, 7))]
    if kind == "sine":
        x = synth.sine_field(shape, seed=seed)
    elif kind == "lognormal":
        x = np.exp(rng.standard_normal(shape) * 1.5).astype(np.float32)
    elif kind == "noise":
        x = rng.standard_normal(shape).astype(np.float32)
    elif kind == "zeros_block":
        x = synth.sine_field(shape, seed=seed)
        sl = tuple(slice(0, max(1, n // 2)) for n in shape)
        x[sl] = 0.0
    elif kind == "signed_zero":
        x = synth.sine_field(shape, seed=seed)
        x[x < 0] = np.float32(-0.0)
    elif kind == "denormal":  # every 7th value a denormal, the range stays normal
        x = synth.sine_field(shape, seed=seed)
        flat = x.reshape(-1)
        flat[::7] = (flat[::7] * np.float32(1e-39)).astype(np.float32)
    else:
        x = np.repeat(rng.standard_normal(max(1, x_len(shape) // 97 + 1)).astype(np.float32), 97)[:x_len(shape)]
        x = x.reshape(shape)
    return kind, np.ascontiguousarray(x, dtype=np.float32)


def x_len(shape):
    return int(np.prod(shape))


def gpu_run(x, eb, mode):
    xt = torch.from_numpy(x).cuda()
    buf = fz.compress(xt, eb, "rel" if mode == O.EB_REL else "abs")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    if info["status"]:
        return info["status"], None, None, None
    y = fz.decompress(buf, x.shape, err=err)
    torch.cuda.synchronize()
    n = int(info["total_bytes"])
    return 0, buf[:n].cpu().numpy(), y.cpu().numpy(), int(err.item())


@pytest.mark.parametrize("case", range(40))
def test_sweep(case):
    rng = np.random.default_rng(7000 + case)
    rank = int(rng.integers(1, 4))
    shape = draw_shape(rng, rank)
    kind, x = draw_field(rng, shape, 7000 + case)
    mode = O.EB_REL if rng.random() < 0.7 else O.EB_ABS
    eb = float(10 ** rng.uniform(-5, -1))
    if mode == O.EB_ABS:
        span = float(np.max(x) - np.min(x))
        eb = eb * (span if span > 0 else 1.0)
        if eb < 1e-37:
            eb = 1e-37
    print("sweep case", case, shape, kind, "rel" if mode == O.EB_REL else "abs", eb, flush=True)
    ref, st = O.compress(x, eb, mode)
    gst, s, y, err = gpu_run(x, eb, mode)
    assert gst == st, (gst, st)
    if st:
        return
    assert s.size == ref.size and np.array_equal(s, ref)
    assert err == 0
    yo, erro = O.decompress(ref, shape)
    assert erro == 0
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))


def test_sweep_escape_cap_and_denormal_range():
    """Noise far above the bound exceeds the escape cap; a field of denormals
    alone in REL mode gives a bound below the smallest normal fp32 (EB_RANGE);
    in ABS mode it compresses."""
    rng = np.random.default_rng(7100)
    noise = (rng.standard_normal((16, 32, 64)) * 1e6).astype(np.float32)
    den = (synth.sine_field((20, 33, 70), seed=7101) * np.float32(1e-39)).astype(np.float32)
    for x, eb, mode, want in ((noise, 0.5, O.EB_ABS, O.ERR_OUTLIER_CAP), (den, 1e-3, O.EB_REL, O.ERR_EB_RANGE),
                              (den, 1e-37, O.EB_ABS, 0)):
        ref, st = O.compress(x, eb, mode)
        gst, s, y, err = gpu_run(x, eb, mode)
        assert st == gst == want
        if st == 0:
            assert np.array_equal(s, ref)
            yo, _ = O.decompress(ref, x.shape)
            assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))
