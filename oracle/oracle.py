"""ctypes wrapper of the ORACLE (``fzo.c``) -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The product library never does.  Arrays are numpy; nothing here
touches a GPU.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

EB_ABS = 0
EB_REL = 1
EB_PWREL = 2
ERR_NONFINITE = 1
ERR_EB_RANGE = 2
ERR_OUTLIER_CAP = 4

_i64p = ctypes.POINTER(ctypes.c_int64)


def build():
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libfzo.so")
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        L.fzo_bound.argtypes = [ctypes.c_int, _i64p]
        L.fzo_bound.restype = ctypes.c_int64
        L.fzo_header_bytes.argtypes = [ctypes.c_int, _i64p]
        L.fzo_header_bytes.restype = ctypes.c_int64
        L.fzo_n_chunks.argtypes = [ctypes.c_int, _i64p]
        L.fzo_n_chunks.restype = ctypes.c_int64
        L.fzo_eb_params.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp]
        L.fzo_eb_params.restype = ctypes.c_int
        L.fzo_prequant.argtypes = [vp, ctypes.c_int64, ctypes.c_float, vp]
        L.fzo_prequant.restype = ctypes.c_int
        L.fzo_prequant_pw.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, vp]
        L.fzo_prequant_pw.restype = ctypes.c_int
        L.fzo_dequant_pw.argtypes = [ctypes.c_int32, ctypes.c_uint32]
        L.fzo_dequant_pw.restype = ctypes.c_float
        L.fzo_code_of.argtypes = [ctypes.c_int32, vp]
        L.fzo_code_of.restype = ctypes.c_int
        L.fzo_delta_of.argtypes = [ctypes.c_uint16]
        L.fzo_delta_of.restype = ctypes.c_int32
        L.fzo_lorenzo_field.argtypes = [vp, ctypes.c_int, _i64p, vp]
        L.fzo_lorenzo_field.restype = ctypes.c_int
        L.fzo_chunk_codes.argtypes = [vp, ctypes.c_int, _i64p, ctypes.c_float, ctypes.c_int64, vp]
        L.fzo_chunk_codes.restype = ctypes.c_int64
        L.fzo_compress.argtypes = [vp, ctypes.c_int, _i64p, ctypes.c_double, ctypes.c_int, vp, ctypes.c_int64,
                                   vp, ctypes.c_int]
        L.fzo_compress.restype = ctypes.c_int64
        L.fzo_decompress.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int, _i64p]
        L.fzo_decompress.restype = ctypes.c_int
        L.fzo_decompress_threads.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int, _i64p, ctypes.c_int]
        L.fzo_decompress_threads.restype = ctypes.c_int
        L.fzo_compress_pred.argtypes = [vp, ctypes.c_int, _i64p, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp,
                                        ctypes.c_int64, vp, ctypes.c_int]
        L.fzo_compress_pred.restype = ctypes.c_int64
        L.fzo_eb_params_f64.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp]
        L.fzo_eb_params_f64.restype = ctypes.c_int
        L.fzo_prequant_f64.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp]
        L.fzo_prequant_f64.restype = ctypes.c_int
        L.fzo_compress_f64.argtypes = [vp, ctypes.c_int, _i64p, ctypes.c_double, ctypes.c_int, vp, ctypes.c_int64,
                                       vp, ctypes.c_int]
        L.fzo_compress_f64.restype = ctypes.c_int64
        L.fzo_decompress_f64.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int, _i64p]
        L.fzo_decompress_f64.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _dims(shape):
    arr = (ctypes.c_int64 * 3)(*(list(shape) + [1] * (3 - len(shape))))
    return len(shape), arr


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def bound(shape):
    r, d = _dims(shape)
    return lib().fzo_bound(r, d)


def header_bytes(shape):
    r, d = _dims(shape)
    return lib().fzo_header_bytes(r, d)


def n_chunks(shape):
    r, d = _dims(shape)
    return lib().fzo_n_chunks(r, d)


def eb_params(x, eb, mode):
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(4, dtype=np.float32)
    st = lib().fzo_eb_params(_ptr(x), x.size, eb, mode, _ptr(out[0:]), _ptr(out[1:]), _ptr(out[2:]), _ptr(out[3:]))
    return dict(ebx2=out[0], inv=out[1], vmin=out[2], vmax=out[3], status=st)


def prequant(x, inv):
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.zeros(x.shape, dtype=np.int32)
    st = lib().fzo_prequant(_ptr(x), x.size, np.float32(inv), _ptr(q))
    return q, st


def prequant_pw(x, step):
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.zeros(x.shape, dtype=np.int32)
    st = lib().fzo_prequant_pw(_ptr(x), x.size, int(step), _ptr(q))
    return q, st


def dequant_pw(q, step):
    return np.float32(lib().fzo_dequant_pw(int(q), int(step)))


def code_of(d):
    c = np.zeros(1, dtype=np.uint16)
    esc = lib().fzo_code_of(int(d), _ptr(c))
    return int(c[0]), bool(esc)


def delta_of(code):
    return lib().fzo_delta_of(int(code))


def lorenzo_field(q):
    q = np.ascontiguousarray(q, dtype=np.int32)
    r, d = _dims(q.shape)
    out = np.zeros(q.shape, dtype=np.int32)
    assert lib().fzo_lorenzo_field(_ptr(q), r, d, _ptr(out)) == 0
    return out


def chunk_codes(x, inv, c):
    x = np.ascontiguousarray(x, dtype=np.float32)
    r, d = _dims(x.shape)
    out = np.zeros(32768, dtype=np.uint16)
    n = lib().fzo_chunk_codes(_ptr(x), r, d, np.float32(inv), c, _ptr(out))
    assert n >= 0
    return out[:n]


def compress(x, eb, mode=EB_REL, threads=1, global_lorenzo=False):
    """Returns (stream bytes as np.uint8, status).  global_lorenzo: predict
    across chunk borders (the field-global Lorenzo predictor)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    r, d = _dims(x.shape)
    cap = lib().fzo_bound(r, d)
    out = np.zeros(cap, dtype=np.uint8)
    st = np.zeros(1, dtype=np.uint32)
    n = lib().fzo_compress_pred(_ptr(x), r, d, float(eb), int(mode), 1 if global_lorenzo else 0, _ptr(out), cap,
                                _ptr(st), int(threads))
    if n < 0:
        raise ValueError("oracle compress failed: %d" % n)
    return out[:n].copy(), int(st[0])


def decompress(stream, shape, threads=1):
    """Returns (float32 array, error code).  threads: OpenMP threads over
    the chunks (1: the sequential reference; the result is the same)."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    r, d = _dims(shape)
    out = np.zeros(shape, dtype=np.float32)
    if threads == 1:
        err = lib().fzo_decompress(_ptr(s), s.size, _ptr(out), r, d)
    else:
        err = lib().fzo_decompress_threads(_ptr(s), s.size, _ptr(out), r, d, int(threads))
    return out, err


def eb_params_f64(x, eb, mode):
    """fp64 bound parameters: dict(status, ebx2, inv, vmin, vmax), all double."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    o = np.zeros(4, dtype=np.float64)
    st = lib().fzo_eb_params_f64(_ptr(x), x.size, float(eb), int(mode), _ptr(o[0:1]), _ptr(o[1:2]), _ptr(o[2:3]),
                                 _ptr(o[3:4]))
    return {"status": st, "ebx2": float(o[0]), "inv": float(o[1]), "vmin": float(o[2]), "vmax": float(o[3])}


def prequant_f64(x, inv):
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.zeros(x.size, dtype=np.int32)
    st = lib().fzo_prequant_f64(_ptr(x), x.size, float(inv), _ptr(q))
    return q.reshape(x.shape), st


def compress_f64(x, eb, mode=EB_REL, threads=1):
    """fp64 input: returns (stream bytes as np.uint8, status)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    r, d = _dims(x.shape)
    cap = lib().fzo_bound(r, d)
    out = np.zeros(cap, dtype=np.uint8)
    st = np.zeros(1, dtype=np.uint32)
    n = lib().fzo_compress_f64(_ptr(x), r, d, float(eb), int(mode), _ptr(out), cap, _ptr(st), int(threads))
    if n < 0:
        raise ValueError("oracle compress failed: %d" % n)
    return out[:n].copy(), int(st[0])


def decompress_f64(stream, shape):
    """Returns (float64 array, error code)."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    r, d = _dims(shape)
    out = np.zeros(shape, dtype=np.float64)
    err = lib().fzo_decompress_f64(_ptr(s), s.size, _ptr(out), r, d)
    return out, err
