"""A seeded sweep of the extra modes on the GPU against the oracle, through
the C ABI: the point-wise relative bound, fp64 input and the field-global
predictor, each on random ranks, extents (chunk boxes plus or minus one,
odd contiguous extents) and value recipes.  The bar is that of the other
parity tests: the oracle's status, and when it is 0 the same stream bytes and
the same reconstruction bits.
"""
import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
from synth import draw_field, draw_shape

pytestmark = pytest.mark.gpu


def run_case(kind, x, eb, mode):
    name = {O.EB_ABS: "abs", O.EB_REL: "rel", O.EB_PWREL: "pwrel"}[mode]
    if kind == "fp64":
        ref, st = O.compress_f64(x, eb, mode)
        dec = O.decompress_f64
        xt = torch.from_numpy(x).cuda()
        buf = fz.compress(xt, eb, name)
        kw = {"dtype": torch.float64}
    else:
        glob = kind == "global"
        ref, st = O.compress(x, eb, mode, global_lorenzo=glob)
        dec = O.decompress
        xt = torch.from_numpy(x).cuda()
        buf = fz.compress(xt, eb, name, global_lorenzo=glob)
        kw = {"global_lorenzo": glob}
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    assert info["status"] == st, (info["status"], st)
    if st:
        return
    n = int(info["total_bytes"])
    s = buf[:n].cpu().numpy()
    assert s.size == ref.size and np.array_equal(s, ref)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, x.shape, err=err, **kw)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    yo, erro = dec(ref, x.shape)
    assert erro == 0
    w = np.uint64 if kind == "fp64" else np.uint32
    assert np.array_equal(y.cpu().numpy().view(w), yo.view(w))


@pytest.mark.parametrize("case", range(36))
def test_sweep_modes(case):
    rng = np.random.default_rng(9000 + case)
    kind = ("pwrel", "fp64", "global")[case % 3]
    rank = int(rng.integers(1, 4))
    shape = draw_shape(rng, rank)
    vkind, x = draw_field(rng, shape, 9000 + case)
    if kind == "pwrel":
        mode, eb = O.EB_PWREL, float(10 ** rng.uniform(-4, -1))
        x = np.abs(x) + np.float32(1e-3)  # positive values: no sign changes to escape
    else:
        mode = O.EB_REL if rng.random() < 0.7 else O.EB_ABS
        eb = float(10 ** rng.uniform(-5, -1))
        if mode == O.EB_ABS:
            span = float(np.max(x) - np.min(x))
            eb = max(eb * (span if span > 0 else 1.0), 1e-37)
        if kind == "fp64":
            x = x.astype(np.float64) * 1.000000123
    print("modes case", case, kind, shape, vkind, mode, eb, flush=True)
    run_case(kind, np.ascontiguousarray(x), eb, mode)
