"""Python binding of libfzmi (the MI355X FZ-GPU hot path).

Argument marshalling only: every step of compression and decompression runs
in the HIP kernels of ``libfzmi.so``.  torch supplies device memory and the
current HIP stream.  If the shared library is missing the import of any
function here raises; there is no CPU fallback.

    s = compress(x, 1e-3)                 # x: float32 CUDA tensor, REL eb
    n = stream_size(s)                    # reads the 128-byte header (syncs)
    y = decompress(s, x.shape)            # float32 CUDA tensor
"""
import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfzmi.so")

FZ_EB_ABS = 0
FZ_EB_REL = 1
FZ_EB_PWREL = 2
STATUS_NONFINITE = 1
STATUS_EB_RANGE = 2
STATUS_OUTLIER_CAP = 4
ERRORS = {0: "ok", 1: "invalid argument", 2: "HIP runtime error", 3: "input holds NaN or Inf",
          4: "error bound out of range", 5: "too many escaped codes", 6: "malformed stream",
          7: "unsupported stream version", 8: "stream carries a compression error"}

_LIB = None


class FzDims(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("n", ctypes.c_uint64 * 3)]


class FzInfo(ctypes.Structure):
    _fields_ = [("version", ctypes.c_uint32), ("status", ctypes.c_uint32), ("rank", ctypes.c_uint32),
                ("eb_mode", ctypes.c_uint32), ("n", ctypes.c_uint64 * 3), ("eb_user", ctypes.c_double),
                ("ebx2", ctypes.c_float), ("inv", ctypes.c_float), ("vmin", ctypes.c_float),
                ("vmax", ctypes.c_float), ("n_chunks", ctypes.c_uint32), ("nnz_blocks", ctypes.c_uint64),
                ("n_outliers", ctypes.c_uint64), ("total_bytes", ctypes.c_uint64),
                ("header_bytes", ctypes.c_uint64), ("dtype", ctypes.c_uint32), ("predictor", ctypes.c_uint32),
                ("ebx2_f64", ctypes.c_double), ("inv_f64", ctypes.c_double)]


class FzCompressJob(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("dims", FzDims), ("eb", ctypes.c_double), ("eb_mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("d_out", ctypes.c_void_p)]


class FzTiming(ctypes.Structure):
    _fields_ = [("range_begin", ctypes.c_void_p), ("main_begin", ctypes.c_void_p), ("main_end", ctypes.c_void_p),
                ("done", ctypes.c_void_p)]


class FzDecompressJob(ctypes.Structure):
    _fields_ = [("d_stream", ctypes.c_void_p), ("dims", FzDims), ("d_out", ctypes.c_void_p),
                ("d_err", ctypes.c_void_p), ("stream_bytes", ctypes.c_uint64)]


class FzRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("eb_mode", ctypes.c_int32), ("eb", ctypes.c_double), ("dims", FzDims),
                ("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p), ("d_err", ctypes.c_void_p),
                ("hbm_bytes", ctypes.c_uint64), ("stream_bytes", ctypes.c_uint64), ("ready_event", ctypes.c_void_p)]


class FzServerReport(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("mean_batch", ctypes.c_double), ("admission_waits", ctypes.c_uint64),
                ("inflight_max_bytes", ctypes.c_uint64), ("input_bytes", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double)]


class FzQuality(ctypes.Structure):
    _fields_ = [("max_abs_err", ctypes.c_double), ("mse", ctypes.c_double), ("psnr", ctypes.c_double),
                ("vmin", ctypes.c_double), ("vmax", ctypes.c_double), ("n", ctypes.c_uint64),
                ("nonfinite", ctypes.c_uint64)]


class FzError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__("%s: %s (%d)" % (what, ERRORS.get(code, "unknown"), code))
        self.code = code


def lib():
    """Load libfzmi.so from the package directory (build it with build.py)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfzmi.so is not built; run `python -m paper_2304_12557_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(FzDims)
        L.fz_compress_bound.argtypes = [dp]
        L.fz_compress_bound.restype = ctypes.c_size_t
        L.fz_header_bytes.argtypes = [dp]
        L.fz_header_bytes.restype = ctypes.c_size_t
        L.fz_stream_bound.argtypes = [dp]
        L.fz_stream_bound.restype = ctypes.c_size_t
        L.fz_compress_noalloc.argtypes = [vp, dp, ctypes.c_double, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.fz_compress_noalloc.restype = ctypes.c_int
        L.fz_compress.argtypes = [vp, dp, ctypes.c_double, ctypes.c_int, vp, vp]
        L.fz_compress.restype = ctypes.c_int
        L.fz_compress_timed.argtypes = [vp, dp, ctypes.c_double, ctypes.c_int, vp, vp, ctypes.POINTER(FzTiming)]
        L.fz_compress_timed.restype = ctypes.c_int
        sz = ctypes.c_size_t
        L.fz_decompress.argtypes = [vp, sz, vp, dp, vp, vp]
        L.fz_decompress.restype = ctypes.c_int
        L.fz_compress_bound_f64.argtypes = [dp]
        L.fz_compress_bound_f64.restype = ctypes.c_size_t
        L.fz_compress_f64.argtypes = [vp, dp, ctypes.c_double, ctypes.c_int, vp, vp]
        L.fz_compress_f64.restype = ctypes.c_int
        L.fz_decompress_f64.argtypes = [vp, sz, vp, dp, vp, vp]
        L.fz_decompress_f64.restype = ctypes.c_int
        L.fz_compress_bound_global.argtypes = [dp]
        L.fz_compress_bound_global.restype = ctypes.c_size_t
        L.fz_compress_global.argtypes = [vp, dp, ctypes.c_double, ctypes.c_int, vp, vp]
        L.fz_compress_global.restype = ctypes.c_int
        L.fz_decompress_global_work_bytes.argtypes = [dp]
        L.fz_decompress_global_work_bytes.restype = ctypes.c_size_t
        L.fz_decompress_global.argtypes = [vp, sz, vp, dp, vp, vp, vp]
        L.fz_decompress_global.restype = ctypes.c_int
        L.fz_stream_info.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(FzInfo)]
        L.fz_stream_info.restype = ctypes.c_int
        L.fz_strerror.argtypes = [ctypes.c_int]
        L.fz_strerror.restype = ctypes.c_char_p
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.fz_batch_create_compress.argtypes = [ctypes.c_int, ctypes.POINTER(FzCompressJob), pp]
        L.fz_batch_create_compress.restype = ctypes.c_int
        L.fz_batch_create_decompress.argtypes = [ctypes.c_int, ctypes.POINTER(FzDecompressJob), pp]
        L.fz_batch_create_decompress.restype = ctypes.c_int
        for name in ("fz_batch_run", "fz_batch_tune"):
            getattr(L, name).argtypes = [vp, vp]
            getattr(L, name).restype = ctypes.c_int
        L.fz_batch_destroy.argtypes = [vp]
        L.fz_batch_destroy.restype = ctypes.c_int
        L.fz_server_create.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, pp]
        L.fz_server_create.restype = ctypes.c_int
        L.fz_server_submit.argtypes = [vp, ctypes.POINTER(FzRequest), ctypes.POINTER(ctypes.c_uint64)]
        L.fz_server_submit.restype = ctypes.c_int
        L.fz_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        L.fz_server_wait.restype = ctypes.c_int
        L.fz_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        L.fz_server_poll.restype = ctypes.c_int
        L.fz_server_stats.argtypes = [vp, ctypes.POINTER(FzServerReport)]
        L.fz_server_stats.restype = ctypes.c_int
        for name in ("fz_server_reset_stats", "fz_server_destroy"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = ctypes.c_int
        L.fz_quality_work_bytes.argtypes = [dp]
        L.fz_quality_work_bytes.restype = ctypes.c_size_t
        L.fz_quality.argtypes = [vp, vp, dp, vp, vp, vp]
        L.fz_quality.restype = ctypes.c_int
        L.fz_abl_pred_quant.argtypes = [ctypes.c_int, vp, dp, ctypes.c_float, vp, vp, vp]
        L.fz_abl_bitshuffle.argtypes = [vp, dp, vp, vp]
        L.fz_abl_mark.argtypes = [vp, dp, vp, vp]
        L.fz_abl_bitshuffle_mark.argtypes = [vp, dp, vp, vp, vp]
        L.fz_abl_bitshuffle_ballot.argtypes = [vp, dp, vp, vp]
        L.fz_abl_bitshuffle_mark_ballot.argtypes = [vp, dp, vp, vp, vp]
        L.fz_abl_encode.argtypes = [vp, vp, dp, vp, vp, vp]
        for name in ("fz_abl_pred_quant", "fz_abl_bitshuffle", "fz_abl_mark", "fz_abl_bitshuffle_mark",
                     "fz_abl_bitshuffle_ballot", "fz_abl_bitshuffle_mark_ballot", "fz_abl_encode"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


SYMBOLS = ["fz_compress_bound", "fz_header_bytes", "fz_stream_bound", "fz_compress_noalloc", "fz_compress", "fz_compress_timed", "fz_decompress", "fz_stream_info", "fz_strerror",
           "fz_batch_create_compress", "fz_batch_create_decompress", "fz_batch_run", "fz_batch_tune",
           "fz_batch_destroy", "fz_server_create", "fz_server_submit", "fz_server_wait", "fz_server_poll",
           "fz_server_stats", "fz_server_reset_stats", "fz_server_destroy", "fz_quality_work_bytes", "fz_quality",
           "fz_abl_pred_quant", "fz_abl_bitshuffle", "fz_abl_mark", "fz_abl_bitshuffle_mark", "fz_abl_encode",
           "fz_abl_bitshuffle_ballot", "fz_abl_bitshuffle_mark_ballot", "fz_compress_bound_f64", "fz_compress_f64", "fz_decompress_f64", "fz_compress_bound_global",
           "fz_compress_global", "fz_decompress_global_work_bytes", "fz_decompress_global"]
FZ_REQ_COMPRESS = 0
FZ_REQ_DECOMPRESS = 1


def dims_of(shape):
    shape = tuple(int(s) for s in shape)
    if not 1 <= len(shape) <= 3:
        raise ValueError("rank must be 1, 2 or 3")
    d = FzDims()
    d.rank = len(shape)
    for i in range(3):
        d.n[i] = shape[i] if i < len(shape) else 1
    return d


def compress_bound(shape, f64=False, global_lorenzo=False):
    """Output bytes ``compress`` needs for a field of this shape (fp32, fp64
    input with ``f64=True``, or the field-global predictor)."""
    fn = (lib().fz_compress_bound_f64 if f64 else
          lib().fz_compress_bound_global if global_lorenzo else lib().fz_compress_bound)
    return int(fn(ctypes.byref(dims_of(shape))))


def header_bytes(shape):
    return int(lib().fz_header_bytes(ctypes.byref(dims_of(shape))))


def stream_bound(shape):
    """Worst-case stream bytes of a field of this shape (no scratch)."""
    return int(lib().fz_stream_bound(ctypes.byref(dims_of(shape))))


def _nbytes(t):
    return t.numel() * t.element_size()


def _check_buffer(t, name, dtypes, align, numel=None):
    """Raise ValueError unless t is a contiguous CUDA tensor of one of
    `dtypes` whose data starts on an `align`-byte boundary (and, if given,
    holds at least `numel` elements): what the C ABI requires of it."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.dtype not in dtypes:
        raise ValueError("%s must be of dtype %s" % (name, " or ".join(str(d) for d in dtypes)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.data_ptr() % align:
        raise ValueError("%s must start on a %d-byte boundary" % (name, align))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s must hold at least %d elements" % (name, numel))


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _mode(mode):
    if mode in ("rel", FZ_EB_REL):
        return FZ_EB_REL
    if mode in ("abs", FZ_EB_ABS):
        return FZ_EB_ABS
    if mode in ("pwrel", FZ_EB_PWREL):
        return FZ_EB_PWREL
    raise ValueError("mode must be 'rel', 'abs' or 'pwrel'")


def compress(x, eb, mode="rel", out=None, stream=None, global_lorenzo=False, events=None):
    """Compress a float32 or float64 CUDA tensor; returns the uint8 output
    buffer (``compress_bound`` bytes; the stream occupies its first
    ``stream_size(buf)`` bytes).  ``global_lorenzo``: the field-global
    predictor (float32 input).  ``events``: a dict of torch.cuda.Event
    objects under any of the keys range_begin, main_begin, main_end, done,
    recorded between the launches (fz_compress_timed; float32 input with the
    chunk-local predictor).  Asynchronous on ``stream``."""
    import torch

    if not (x.is_cuda and x.dtype in (torch.float32, torch.float64) and x.is_contiguous()):
        raise ValueError("x must be a contiguous float32 or float64 CUDA tensor")
    f64 = x.dtype == torch.float64
    if f64 and global_lorenzo:
        raise ValueError("the field-global predictor takes float32 input")
    dims = dims_of(x.shape)
    bound = compress_bound(x.shape, f64=f64, global_lorenzo=global_lorenzo)
    if out is None:
        out = torch.empty(bound, dtype=torch.uint8, device=x.device)
    else:
        _check_buffer(out, "out", (torch.uint8,), 256, bound)
    if events:
        if f64 or global_lorenzo:
            raise ValueError("events are recorded for float32 input with the chunk-local predictor")
        t = FzTiming()
        for k, ev in events.items():
            if ev is not None:
                ev.record(stream if stream is not None else torch.cuda.current_stream())  # creates the event
                setattr(t, k, ev.cuda_event)
        rc = lib().fz_compress_timed(ctypes.c_void_p(x.data_ptr()), ctypes.byref(dims), float(eb), _mode(mode),
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream), ctypes.byref(t))
        if rc:
            raise FzError(rc, "fz_compress_timed")
        return out
    fn = lib().fz_compress_f64 if f64 else lib().fz_compress_global if global_lorenzo else lib().fz_compress
    rc = fn(ctypes.c_void_p(x.data_ptr()), ctypes.byref(dims), float(eb), _mode(mode),
            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    if rc:
        raise FzError(rc, "fz_compress")
    return out


def compress_noalloc(x, eb, mode="rel", out=None, stream=None):
    """fz_compress_noalloc: compress a float32 CUDA tensor with the
    library's own scratch array; ``out`` (uint8, 256-byte aligned) needs only
    ``stream_bound`` bytes.  The call allocates nothing when ``out`` is given.
    Asynchronous on ``stream``; calls that overlap on one device race."""
    import torch

    if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise ValueError("x must be a contiguous float32 CUDA tensor")
    dims = dims_of(x.shape)
    need = stream_bound(x.shape)
    if out is None:
        out = torch.empty(need, dtype=torch.uint8, device=x.device)
    else:
        _check_buffer(out, "out", (torch.uint8,), 256, need)
    rc = lib().fz_compress_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.byref(dims), float(eb), _mode(mode),
                                   ctypes.c_void_p(out.data_ptr()), _nbytes(out), _stream_ptr(stream))
    if rc:
        raise FzError(rc, "fz_compress_noalloc")
    return out


def decompress(s, shape, out=None, err=None, stream=None, dtype=None, global_lorenzo=False, work=None):
    """Decompress a stream held in a uint8 CUDA tensor into float32, or into
    float64 for a stream of fp64 input (``dtype=torch.float64``, or an
    ``out`` of that type).  If ``err`` (a 1-element int32 CUDA tensor) is
    given it receives 0 or the error code of a stream rejected on the
    device."""
    import torch

    dims = dims_of(shape)
    _check_buffer(s, "s", (torch.uint8,), 256, header_bytes(shape))
    if err is not None:
        _check_buffer(err, "err", (torch.int32,), 4, 1)
    if dtype is None:
        dtype = out.dtype if out is not None else torch.float32
    if dtype not in (torch.float32, torch.float64):
        raise ValueError("dtype must be float32 or float64")
    if out is None:
        out = torch.empty(tuple(shape), dtype=dtype, device=s.device)
    elif out.dtype != dtype or not out.is_cuda or not out.is_contiguous() or out.numel() != math.prod(shape):
        raise ValueError("out must be a contiguous %s CUDA tensor of the field's size" % dtype)
    errp = ctypes.c_void_p(err.data_ptr() if err is not None else 0)
    if global_lorenzo:  # a stream of the field-global predictor (header byte 15 = 1)
        if dtype != torch.float32:
            raise ValueError("the field-global predictor takes float32 fields")
        nwork = int(lib().fz_decompress_global_work_bytes(ctypes.byref(dims)))
        if work is None:  # freed when this returns: keep it until the launch's stream has passed it
            work = torch.empty(max(nwork, 16), dtype=torch.uint8, device=s.device)
            work.record_stream(stream if stream is not None else torch.cuda.current_stream())
        elif _nbytes(work) < nwork or not work.is_cuda or not work.is_contiguous() or work.data_ptr() % 256:
            raise ValueError("work must be a contiguous CUDA tensor of at least %d bytes on a 256-byte boundary"
                             % nwork)
        rc = lib().fz_decompress_global(ctypes.c_void_p(s.data_ptr()), _nbytes(s), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.byref(dims), errp, ctypes.c_void_p(work.data_ptr()),
                                        _stream_ptr(stream))
    else:
        fn = lib().fz_decompress_f64 if dtype == torch.float64 else lib().fz_decompress
        rc = fn(ctypes.c_void_p(s.data_ptr()), _nbytes(s), ctypes.c_void_p(out.data_ptr()), ctypes.byref(dims), errp,
                _stream_ptr(stream))
    if rc:
        raise FzError(rc, "fz_decompress")
    return out


def quality(x, y, stream=None):
    """Distortion of y against x (float32 CUDA tensors of one shape, rank 1-3)
    computed by the library's kernels; returns a dict with max_abs_err, mse,
    psnr (dB), vmin, vmax, n, nonfinite.  Synchronizes the stream."""
    import torch

    for name, t in (("x", x), ("y", y)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)
    if tuple(x.shape) != tuple(y.shape):
        raise ValueError("x and y differ in shape")
    dims = dims_of(x.shape)
    nwork = int(lib().fz_quality_work_bytes(ctypes.byref(dims)))
    if nwork == 0:
        raise FzError(1, "fz_quality_work_bytes")
    work = torch.empty(nwork, dtype=torch.uint8, device=x.device)
    res = torch.empty(ctypes.sizeof(FzQuality), dtype=torch.uint8, device=x.device)
    rc = lib().fz_quality(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), ctypes.byref(dims),
                          ctypes.c_void_p(res.data_ptr()), ctypes.c_void_p(work.data_ptr()), _stream_ptr(stream))
    if rc:
        raise FzError(rc, "fz_quality")
    q = FzQuality.from_buffer_copy(bytes(res.cpu().numpy().tobytes()))
    return {f: getattr(q, f) for f, _ in FzQuality._fields_}


class Ablation:
    """The paper's per-kernel ablation pipeline (fz_abl_* in fz.h) on one 3-D
    float32 CUDA tensor whose extents are multiples of 16 x 32 x 64; owns the
    intermediate buffers.  Each method enqueues one stage on ``stream``."""

    def __init__(self, x):
        import torch

        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 3):
            raise ValueError("x must be a contiguous 3-D float32 CUDA tensor")
        self.x, self.dims = x, dims_of(x.shape)
        n = x.numel()
        dev = x.device
        self.codes = torch.empty(n, dtype=torch.int16, device=dev)
        self.outliers = torch.empty(n, dtype=torch.int32, device=dev)
        self.tiles = torch.empty(n // 2, dtype=torch.int32, device=dev)
        self.steps = n // 2048
        self.flags = torch.empty(self.steps * 4, dtype=torch.int64, device=dev)
        self.offsets = torch.empty(self.steps + 1, dtype=torch.int64, device=dev)
        self.out = torch.empty(n * 2, dtype=torch.uint8, device=dev)

    def _call(self, rc, what):
        if rc:
            raise FzError(rc, what)

    def pred_quant(self, version, inv, stream=None):
        self._call(lib().fz_abl_pred_quant(int(version), ctypes.c_void_p(self.x.data_ptr()), ctypes.byref(self.dims),
                                           float(inv), ctypes.c_void_p(self.codes.data_ptr()),
                                           ctypes.c_void_p(self.outliers.data_ptr()), _stream_ptr(stream)),
                   "fz_abl_pred_quant")

    def bitshuffle(self, stream=None, ballot=False):
        name = "fz_abl_bitshuffle_ballot" if ballot else "fz_abl_bitshuffle"
        self._call(getattr(lib(), name)(ctypes.c_void_p(self.codes.data_ptr()), ctypes.byref(self.dims),
                                        ctypes.c_void_p(self.tiles.data_ptr()), _stream_ptr(stream)), name)

    def mark(self, stream=None):
        self._call(lib().fz_abl_mark(ctypes.c_void_p(self.tiles.data_ptr()), ctypes.byref(self.dims),
                                     ctypes.c_void_p(self.flags.data_ptr()), _stream_ptr(stream)), "fz_abl_mark")

    def bitshuffle_mark(self, stream=None, ballot=False):
        name = "fz_abl_bitshuffle_mark_ballot" if ballot else "fz_abl_bitshuffle_mark"
        self._call(getattr(lib(), name)(ctypes.c_void_p(self.codes.data_ptr()), ctypes.byref(self.dims),
                                        ctypes.c_void_p(self.tiles.data_ptr()),
                                        ctypes.c_void_p(self.flags.data_ptr()), _stream_ptr(stream)), name)

    def encode(self, stream=None):
        self._call(lib().fz_abl_encode(ctypes.c_void_p(self.tiles.data_ptr()), ctypes.c_void_p(self.flags.data_ptr()),
                                       ctypes.byref(self.dims), ctypes.c_void_p(self.offsets.data_ptr()),
                                       ctypes.c_void_p(self.out.data_ptr()), _stream_ptr(stream)), "fz_abl_encode")


def stream_info(header):
    """Parse the header from host bytes (or a CUDA tensor, which is copied)."""
    if hasattr(header, "is_cuda"):
        header = header[:128].cpu().numpy().tobytes()
    buf = (ctypes.c_uint8 * len(header)).from_buffer_copy(bytes(header))
    info = FzInfo()
    rc = lib().fz_stream_info(ctypes.cast(buf, ctypes.c_void_p), len(header), ctypes.byref(info))
    if rc:
        raise FzError(rc, "fz_stream_info")
    return {f: (list(getattr(info, f)) if f == "n" else getattr(info, f)) for f, _ in FzInfo._fields_}


def stream_size(buf):
    """Total stream bytes, read from the header of a compressed buffer."""
    return int(stream_info(buf)["total_bytes"])


class Batch:
    """A plan over many fields (libfzmi's batch layer): ``run()`` enqueues the
    whole batch in a fixed number of launches, capturable in a graph.

    Compression: ``Batch.compress([(x, eb, mode, out), ...])`` with float32
    CUDA tensors ``x`` and uint8 CUDA tensors ``out`` of ``compress_bound``
    bytes (``out=None`` allocates one).  Decompression:
    ``Batch.decompress([(stream, shape, out, err), ...])``.  The tensors are
    kept referenced by the plan."""

    def __init__(self, handle, tensors, outs):
        self._h = ctypes.c_void_p(handle)
        self._tensors = tensors
        self.outs = outs

    @classmethod
    def compress(cls, jobs):
        import torch

        arr = (FzCompressJob * len(jobs))()
        keep, outs = [], []
        for i, (x, eb, mode, out) in enumerate(jobs):
            if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
                raise ValueError("job %d: x must be a contiguous float32 CUDA tensor" % i)
            dims = dims_of(x.shape)
            bound = int(lib().fz_compress_bound(ctypes.byref(dims)))
            if out is None:
                out = torch.empty(bound, dtype=torch.uint8, device=x.device)
            else:
                _check_buffer(out, "job %d: out" % i, (torch.uint8,), 256, bound)
            arr[i].d_in, arr[i].dims, arr[i].eb = x.data_ptr(), dims, float(eb)
            arr[i].eb_mode, arr[i].d_out = _mode(mode), out.data_ptr()
            keep += [x, out]
            outs.append(out)
        h = ctypes.c_void_p()
        rc = lib().fz_batch_create_compress(len(jobs), arr, ctypes.byref(h))
        if rc:
            raise FzError(rc, "fz_batch_create_compress")
        return cls(h.value, keep, outs)

    @classmethod
    def decompress(cls, jobs):
        import torch

        arr = (FzDecompressJob * len(jobs))()
        keep, outs = [], []
        for i, (s, shape, out, err) in enumerate(jobs):
            _check_buffer(s, "job %d: stream" % i, (torch.uint8,), 256, header_bytes(shape))
            if out is None:
                out = torch.empty(tuple(shape), dtype=torch.float32, device=s.device)
            else:
                _check_buffer(out, "job %d: out" % i, (torch.float32,), 4, math.prod(shape))
            if err is not None:
                _check_buffer(err, "job %d: err" % i, (torch.int32,), 4, 1)
            arr[i].d_stream, arr[i].dims, arr[i].d_out = s.data_ptr(), dims_of(shape), out.data_ptr()
            arr[i].d_err = err.data_ptr() if err is not None else None
            arr[i].stream_bytes = _nbytes(s)
            keep += [s, out] + ([err] if err is not None else [])
            outs.append(out)
        h = ctypes.c_void_p()
        rc = lib().fz_batch_create_decompress(len(jobs), arr, ctypes.byref(h))
        if rc:
            raise FzError(rc, "fz_batch_create_decompress")
        return cls(h.value, keep, outs)

    def run(self, stream=None):
        rc = lib().fz_batch_run(self._h, _stream_ptr(stream))
        if rc:
            raise FzError(rc, "fz_batch_run")
        return self.outs

    def tune(self, stream=None):
        rc = lib().fz_batch_tune(self._h, _stream_ptr(stream))
        if rc:
            raise FzError(rc, "fz_batch_tune")

    def close(self):
        if self._h is not None and self._h.value:
            lib().fz_batch_destroy(self._h)
        self._h = None
        self._tensors = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request server (continuous batching with HBM admission) on the
    current device.  ``submit_compress`` / ``submit_decompress`` queue a
    request and return a ticket; ``wait(ticket)`` blocks until it is done and
    returns its output tensor.  Request tensors stay referenced until then."""

    def __init__(self, hbm_budget, slots=4, max_batch=64):
        h = ctypes.c_void_p()
        rc = lib().fz_server_create(int(hbm_budget), int(slots), int(max_batch), ctypes.byref(h))
        if rc:
            raise FzError(rc, "fz_server_create")
        self._h = h
        self._live = {}

    def _submit(self, req, keep, out):
        import torch

        # the request's kernels wait (on the device) for what the current
        # stream has enqueued so far: the producer of the input, and any
        # earlier use of the output's memory
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        req.ready_event = ev.cuda_event
        t = ctypes.c_uint64()
        rc = lib().fz_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if rc:
            raise FzError(rc, "fz_server_submit")
        self._live[t.value] = (keep + [ev], out)
        return t.value

    def submit_compress(self, x, eb, mode="rel", out=None, hbm_bytes=0):
        import torch

        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
            raise ValueError("x must be a contiguous float32 CUDA tensor")
        dims = dims_of(x.shape)
        bound = int(lib().fz_compress_bound(ctypes.byref(dims)))
        if out is None:
            out = torch.empty(bound, dtype=torch.uint8, device=x.device)
        else:
            _check_buffer(out, "out", (torch.uint8,), 256, bound)
        r = FzRequest(kind=FZ_REQ_COMPRESS, eb_mode=_mode(mode), eb=float(eb), dims=dims, d_in=x.data_ptr(),
                      d_out=out.data_ptr(), d_err=None, hbm_bytes=int(hbm_bytes))
        return self._submit(r, [x, out], out)

    def submit_decompress(self, s, shape, out=None, err=None, hbm_bytes=0):
        import torch

        _check_buffer(s, "s", (torch.uint8,), 256, header_bytes(shape))
        if out is None:
            out = torch.empty(tuple(shape), dtype=torch.float32, device=s.device)
        else:
            _check_buffer(out, "out", (torch.float32,), 4, math.prod(shape))
        if err is not None:
            _check_buffer(err, "err", (torch.int32,), 4, 1)
        r = FzRequest(kind=FZ_REQ_DECOMPRESS, eb_mode=0, eb=0.0, dims=dims_of(shape), d_in=s.data_ptr(),
                      d_out=out.data_ptr(), d_err=err.data_ptr() if err is not None else None,
                      hbm_bytes=int(hbm_bytes), stream_bytes=_nbytes(s))
        return self._submit(r, [s, out, err], out)

    def wait(self, ticket):
        st = ctypes.c_int()
        rc = lib().fz_server_wait(self._h, int(ticket), ctypes.byref(st))
        if rc:
            raise FzError(rc, "fz_server_wait")
        _, out = self._live.pop(ticket)
        if st.value:
            raise FzError(st.value, "request %d" % ticket)
        return out

    def done(self, ticket):
        d = ctypes.c_int()
        rc = lib().fz_server_poll(self._h, int(ticket), ctypes.byref(d))
        if rc:
            raise FzError(rc, "fz_server_poll")
        return bool(d.value)

    def stats(self):
        r = FzServerReport()
        rc = lib().fz_server_stats(self._h, ctypes.byref(r))
        if rc:
            raise FzError(rc, "fz_server_stats")
        return {f: getattr(r, f) for f, _ in FzServerReport._fields_}

    def reset_stats(self):
        lib().fz_server_reset_stats(self._h)

    def close(self):
        if self._h is not None and self._h.value:
            lib().fz_server_destroy(self._h)
        self._h = None
        self._live = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
