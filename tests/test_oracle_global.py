"""Pins of the oracle's field-global Lorenzo predictor (CPU only).

The global predictor applies the Lorenzo difference over the whole field
(zero outside the field) instead of inside each chunk; the deltas are coded
per chunk as before and header byte 15 records the choice.  The pins: a field
of one chunk gives the chunk-local stream but for that byte; a constant field
stores its one nonzero delta once instead of once per chunk; the independent
numpy reader's chunk-local sums of the stored deltas equal the
inclusion-exclusion of q over each chunk's lower faces (a formula of its own,
not the oracle's); every stage stays lossless, so both predictors
reconstruct the same values; a stream with an unknown predictor byte is
rejected.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
import stream_np
import synth

BOX = {1: (32768,), 2: (32, 1024), 3: (16, 32, 64)}


@pytest.mark.parametrize("shape", [(16, 32, 64), (9, 20, 33), (32, 1024), (7, 900), (32768,), (1000,)])
def test_one_chunk_equals_the_chunk_local_stream(shape):
    x = synth.sine_field(shape, seed=len(shape))
    sl, st1 = O.compress(x, 1e-3, O.EB_REL)
    sg, st2 = O.compress(x, 1e-3, O.EB_REL, global_lorenzo=True)
    assert st1 == st2 == 0 and sl.size == sg.size
    assert np.nonzero(sl != sg)[0].tolist() == [15] and sg[15] == 1


@pytest.mark.parametrize("shape", [(40, 70, 130), (70, 2100), (100000,)])
def test_constant_field_one_delta_per_field(shape):
    x = np.full(shape, 5.0, dtype=np.float32)  # q = 5 everywhere at eb = 1/2
    sl, _ = O.compress(x, 0.5, O.EB_ABS)
    sg, _ = O.compress(x, 0.5, O.EB_ABS, global_lorenzo=True)
    hl, hg = stream_np.header(sl), stream_np.header(sg)
    # code 5 sets planes 0 and 2 of the brick holding the origin cell
    assert hg["nnz"] == 2 and hl["nnz"] == 2 * hl["n_chunks"]


def face_sum(q, box):
    """p = sum over subsets S of the axes of (-1)^|S| q(coordinates in S moved
    to the plane just before the chunk's origin), a ghost counting 0."""
    q = q.astype(np.int64)
    rank = q.ndim
    p = np.zeros(q.shape, dtype=np.int64)
    idx = np.indices(q.shape)
    for S in itertools.product((0, 1), repeat=rank):
        coords, ok = [], np.ones(q.shape, dtype=bool)
        for a in range(rank):
            c = idx[a]
            if S[a]:
                c = (c // box[a]) * box[a] - 1
                ok &= c >= 0
            coords.append(np.where(c >= 0, c, 0))
        term = np.where(ok, q[tuple(coords)], 0)
        p += (-1) ** sum(S) * term
    return (p & 0xFFFFFFFF).astype(np.uint32).view(np.int32)


@pytest.mark.parametrize("shape,eb", [((40, 70, 130), 1e-3), ((70, 2100), 1e-3), ((100000,), 1e-4),
                                      ((17, 33, 65), 1e-2)])
def test_reader_matches_face_inclusion_exclusion(shape, eb):
    x = synth.sine_field(shape, seed=sum(shape))
    sg, st = O.compress(x, eb, O.EB_REL, global_lorenzo=True)
    assert st == 0
    h = stream_np.header(sg)
    q, qst = O.prequant(x, h["inv"])
    assert qst == 0
    got = stream_np.read(sg, shape)["q"]
    assert np.array_equal(got, face_sum(q.reshape(shape), BOX[len(shape)]))


@pytest.mark.parametrize("shape,mode,eb", [((40, 70, 130), O.EB_REL, 1e-3), ((70, 2100), O.EB_ABS, 1e-3),
                                           ((100000,), O.EB_REL, 1e-4), ((20, 40, 70), O.EB_PWREL, 1e-2)])
def test_both_predictors_reconstruct_the_same_values(shape, mode, eb):
    x = synth.wide_field(shape, seed=3) if mode == O.EB_PWREL else synth.sine_field(shape, seed=3)
    sl, st1 = O.compress(x, eb, mode)
    sg, st2 = O.compress(x, eb, mode, global_lorenzo=True)
    assert st1 == st2 == 0
    yl, e1 = O.decompress(sl, shape)
    yg, e2 = O.decompress(sg, shape)
    assert e1 == e2 == 0
    assert np.array_equal(yl.view(np.uint32), yg.view(np.uint32))


def test_unknown_predictor_byte_is_rejected():
    x = synth.sine_field((20, 40, 70), seed=1)
    s, _ = O.compress(x, 1e-3, O.EB_REL, global_lorenzo=True)
    s = s.copy()
    s[15] = 2
    assert O.decompress(s, x.shape)[1] != 0
