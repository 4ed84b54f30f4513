"""GPU parity of chunks cut by the field's edge, against the oracle.

Such a chunk is loaded like an interior one: its cells outside the field read
other chunks' values, or zeros past the field's end, and their codes are
cleared after the layer.  Their deltas can be large: a field far from zero
(an offset of 10^4 at an absolute bound of 10^-3 gives quantized values near
5 * 10^6) next to the zeros past its end makes the fast pass report escapes
that only cells outside the field need.  The layer then takes the logging
pass, which zeroes those deltas before it looks for escapes, so the stream
must not carry them.  Cases: the three ranks, cut in every dimension, with a
large positive and a large negative offset, plus a field whose last chunk
holds a single cell; the whole stream byte for byte and the reconstruction
bit for bit.
"""
import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu


def run(x, eb, mode):
    print("case", x.shape, eb, mode, flush=True)
    ref, st = O.compress(x, eb, mode)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    buf = fz.compress(xt, eb, "abs" if mode == O.EB_ABS else "rel")
    torch.cuda.synchronize()
    info = fz.stream_info(buf)
    assert info["status"] == st, (info["status"], st)
    n = fz.stream_size(buf)
    s = buf[:n].cpu().numpy()
    assert s.size == ref.size and np.array_equal(s, ref)
    if st:
        return info
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = fz.decompress(buf, x.shape, err=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    yo, e = O.decompress(ref, x.shape)
    assert e == 0
    assert np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32))
    return info


@pytest.mark.parametrize("shape", [(37, 70, 130), (17, 33, 65), (75, 2050), (33, 1025), (100_001,), (32_769,)])
@pytest.mark.parametrize("offset", [1.0e4, -2.5e4])
def test_offset_field_abs(shape, offset):
    x = (synth.sine_field(shape, seed=9000 + len(shape)) + np.float32(offset)).astype(np.float32)
    info = run(x, 1e-3, O.EB_ABS)
    assert info["status"] == 0


@pytest.mark.parametrize("shape", [(37, 70, 130), (75, 2050), (100_001,)])
def test_offset_field_rel(shape):
    # relative bound on a field with a large offset: the range is small, so
    # the quantized values are large and so are the outside cells' deltas
    x = (synth.sine_field(shape, seed=9100 + len(shape)) + np.float32(3.0e3)).astype(np.float32)
    run(x, 1e-4, O.EB_REL)
