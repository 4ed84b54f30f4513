"""The ablation pipeline's kernels on the GPU against the ablation oracle,
stage by stage (all integer outputs: exact equality), for both code versions,
both bitshuffle-mark variants and both transposes (in registers, and by wave
votes as in Sec. 3.3)."""
import numpy as np
import pytest
import torch

import paper_2304_12557_amd as fz
from oracle import ablation as A
from oracle import oracle as O
import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,seed,eb", [((32, 64, 128), 1, 1e-3), ((16, 96, 192), 2, 1e-4), ((48, 32, 64), 3, 1e-2), ((16, 32, 128), 4, 2e-6)])
def test_stages_match_oracle(shape, seed, eb):
    x = synth.sine_field(shape, seed=seed)
    inv = float(O.eb_params(x, eb, O.EB_REL)["inv"])
    print("ablation", shape, eb, flush=True)
    ab = fz.Ablation(torch.from_numpy(x).cuda())
    c1, o1 = A.pred_quant_v1(x, inv)
    c2 = A.pred_quant_v2(x, inv)
    for version, codes in ((1, c1), (2, c2)):
        ab.pred_quant(version, inv)
        torch.cuda.synchronize()
        got = ab.codes.cpu().numpy().view(np.uint16)
        assert np.array_equal(got, codes.reshape(-1)), version
        if version == 1:
            assert np.array_equal(ab.outliers.cpu().numpy(), o1.reshape(-1))
        tiles = A.bitshuffle(codes.reshape(shape))
        flags = A.mark(tiles)
        offsets, payload = A.encode(tiles, flags)
        ab.bitshuffle()
        ab.mark()
        torch.cuda.synchronize()
        assert np.array_equal(ab.tiles.cpu().numpy().view(np.uint32), tiles.reshape(-1)), version
        assert np.array_equal(ab.flags.cpu().numpy().view(np.uint64), flags.reshape(-1)), version
        ab.tiles.zero_()
        ab.flags.zero_()
        ab.bitshuffle_mark()
        ab.encode()
        torch.cuda.synchronize()
        assert np.array_equal(ab.tiles.cpu().numpy().view(np.uint32), tiles.reshape(-1)), version
        assert np.array_equal(ab.flags.cpu().numpy().view(np.uint64), flags.reshape(-1)), version
        # the same stages with the transpose done by wave votes (Sec. 3.3)
        for fused in (False, True):
            ab.tiles.zero_()
            ab.flags.zero_()
            if fused:
                ab.bitshuffle_mark(ballot=True)
            else:
                ab.bitshuffle(ballot=True)
                ab.mark()
            torch.cuda.synchronize()
            assert np.array_equal(ab.tiles.cpu().numpy().view(np.uint32), tiles.reshape(-1)), (version, fused)
            assert np.array_equal(ab.flags.cpu().numpy().view(np.uint64), flags.reshape(-1)), (version, fused)
        got_off = ab.offsets.cpu().numpy().view(np.uint64)
        assert np.array_equal(got_off, offsets), version
        n = int(offsets[-1]) * 16
        assert np.array_equal(ab.out[:n].cpu().numpy(), payload), version
