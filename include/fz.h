/*
 * fz.h -- C ABI of libfzmi, an MI355X (gfx950) implementation of the FZ-GPU
 * compression hot path:
 *   dual-quantization (prequantize to the 2*eb grid, then Lorenzo prediction
 *   on the integers), 16-bit sign-magnitude codes, bitshuffle, and the
 *   zero-block encoder (flags, device-wide prefix sum, compaction), plus the
 *   matching decompressor.
 *
 * Paper: Zhang et al., "FZ-GPU: A Fast and High-Ratio Lossy Compressor for
 * Scientific Computing Applications on GPUs", HPDC'23.  The problem statement
 * (Sec. 2.4) fixes the setting: the field is produced in GPU memory and
 * compressed there; the compressed bytes either stay in GPU memory for a
 * later GPU decompression or are copied out.  Input is fp32 (Sec. 4.1,
 * Table 1); the error bound is absolute or relative to the value range
 * (Sec. 4.1).
 *
 * Conventions for every call:
 *   - pointers named d_* are device pointers (HIP device memory of the
 *     current device); h_* are host pointers;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     calls only enqueue work on it and never synchronize the host;
 *   - the caller owns every buffer; the library allocates nothing per call
 *     and keeps no state between calls; calls on different streams are
 *     independent as long as their buffers do not overlap;
 *   - argument errors return a nonzero fz_status immediately and enqueue
 *     nothing; data-dependent errors are reported on the device (see each
 *     call);
 *   - alignment: a buffer the library writes or reads as a whole (d_out of
 *     the compression calls, d_stream, d_work) must start on a 256-byte
 *     boundary, d_err on a 4-byte boundary and d_res on an 8-byte boundary
 *     (the kernels use atomics and 8- and 16-byte accesses at fixed offsets
 *     in them); inputs and outputs of field values may have any 4-byte (fp32)
 *     or 8-byte (fp64) alignment.  A misaligned pointer is FZ_ERR_ARG.
 */
#ifndef FZ_H
#define FZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FZ_OK = 0,
    FZ_ERR_ARG = 1,          /* invalid argument (returned immediately) */
    FZ_ERR_HIP = 2,          /* a HIP runtime call failed */
    FZ_ERR_NONFINITE = 3,    /* input holds NaN or Inf */
    FZ_ERR_EB_RANGE = 4,     /* error bound unusable: 2*eb not a normal fp32, or |x/(2eb)| >= 2^31;
                              * FZ_EB_PWREL: the step (see fz_compress) outside [2, 2^24) */
    FZ_ERR_OUTLIER_CAP = 5,  /* more than 1024 escaped codes in one chunk of 32768 codes */
    FZ_ERR_STREAM = 6,       /* malformed or inconsistent stream */
    FZ_ERR_VERSION = 7,      /* unknown stream version */
    FZ_ERR_STATUS = 8        /* stream carries a nonzero compression status */
} fz_status;

/* FZ_EB_PWREL: point-wise relative bound (see fz_compress). */
typedef enum { FZ_EB_ABS = 0, FZ_EB_REL = 1, FZ_EB_PWREL = 2 } fz_eb_mode;

/* Field extents, slowest-varying first (a 3-D field 100 x 500 x 500 has
 * n = {100, 500, 500}; x is the contiguous dimension).  rank is 1, 2 or 3;
 * n[rank..2] are ignored.  Limits (beyond them every call rejects the dims
 * with FZ_ERR_ARG, and fz_compress_bound returns 0): every extent in
 * 1 .. 2^40; for rank 2 and 3 the contiguous extent below 2^25; fewer than
 * 2^31 chunks (chunk boxes 16x32x64, 32x1024, 32768); the stream's payload
 * below 64 GiB (offsets are 32-bit in 16-byte units; a larger payload sets
 * FZ_STATUS_BIT_INTERNAL). */
typedef struct {
    uint32_t rank;
    uint32_t reserved;
    uint64_t n[3];
} fz_dims;

/* Parsed stream header (host side). */
typedef struct {
    uint32_t version;
    uint32_t status;      /* OR of FZ_STATUS_BIT_* set during compression */
    uint32_t rank;
    uint32_t eb_mode;
    uint64_t n[3];
    double eb_user;
    float ebx2;           /* fp32(2 * absolute error bound); FZ_EB_PWREL: the step S */
    float inv;            /* fp32(1 / ebx2); FZ_EB_PWREL: 0 */
    float vmin, vmax;     /* value range (REL mode; 0 in ABS mode) */
    uint32_t n_chunks;
    uint64_t nnz_blocks;  /* nonzero 16-byte blocks stored */
    uint64_t n_outliers;  /* escaped codes stored as (index, value) pairs */
    uint64_t total_bytes; /* stream size */
    uint64_t header_bytes;/* header + chunk table + flags */
    uint32_t dtype;       /* input type: 0 fp32, 1 fp64 */
    uint32_t predictor;   /* Lorenzo predictor: 0 inside each chunk, 1 over the whole field */
    double ebx2_f64;      /* fp64 streams: 2 * absolute error bound, in double (0 for fp32) */
    double inv_f64;       /* fp64 streams: 1 / ebx2_f64 (0 for fp32) */
} fz_info;

/* status bits written into the header by the device */
#define FZ_STATUS_BIT_NONFINITE 1u
#define FZ_STATUS_BIT_EB_RANGE 2u
#define FZ_STATUS_BIT_OUTLIER_CAP 4u
#define FZ_STATUS_BIT_INTERNAL 0x80000000u /* a consistency check of the library failed: the stream is invalid */

/* Bytes the caller must provide as d_out of fz_compress: the worst-case
 * stream (every data block nonzero plus the escape cap), then the scratch:
 * chunk tickets and sizes, partial value ranges, and the staging slots in
 * which each compression workgroup assembles a chunk's payload until the
 * chunk's offset is known (one slot of the worst-case chunk payload per
 * chunk, at most 768 slots).  About 0.67 times the input bytes for a
 * 512^3 field, 1.2 times for 64^3; a field smaller than one chunk needs the
 * bound of one chunk (about 180 KB).  0 on invalid dims. */
size_t fz_compress_bound(const fz_dims *dims);

/* Bytes of header + chunk table + flags; depends only on the dims. */
size_t fz_header_bytes(const fz_dims *dims);

/* Worst-case size of a stream (every data block nonzero plus the escape cap
 * of every chunk), without any scratch: about 0.56 times the input bytes.
 * 0 on invalid dims. */
size_t fz_stream_bound(const fz_dims *dims);

/* fz_compress -- the compression pipeline of Sec. 3 (one read of the input;
 * REL mode first reads it once more for the value range).
 *   d_in   : N fp32 values, row-major, slowest-first dims (device, read only)
 *   dims   : host pointer
 *   eb     : absolute error bound (FZ_EB_ABS), bound relative to the value
 *            range max-min (FZ_EB_REL, Sec. 4.1), or point-wise relative
 *            bound eps (FZ_EB_PWREL, below); must be finite and > 0
 *   d_out  : device buffer of at least fz_compress_bound(dims) bytes; on
 *            completion it starts with the stream, whose size is the header's
 *            total_bytes field (little-endian u64 at byte 96)
 * Every reconstructed value differs from the input by at most the error bound
 * (Sec. 2.3 inequality) up to fp32 rounding of x/(2eb) and of q*2eb.
 * FZ_EB_PWREL (the point-wise relative mode, an extension of Sec. 2.3 to a
 * transformed field): the pipeline runs on T(x) = sign(x) * (bits of |x|),
 * an exact integer piecewise-linear log2, with the step S = floor(eps *
 * 2^24 / (1 + eps)) in place of 2eb, q = sign(x) * floor((T + S/2) / S); the
 * reconstruction is the float with bits min(|q| * S, largest finite) and q's
 * sign, so |x' - x| <= eps * max(|x|, 2^-126) for every value, in integer
 * arithmetic with no rounding.  S must lie in [2, 2^24) (eps from about
 * 1.2e-7 to any larger value), else FZ_ERR_EB_RANGE at once.  A sign change
 * between neighbours is a large difference of T and costs an escape, so
 * fields that cross zero often may hit the escape cap; -0 comes back as +0.
 * Data-dependent errors (NaN/Inf, |x/(2eb)| >= 2^31, escape cap) set bits of
 * the header's status word (u32 at byte 8); the rest of the stream is then
 * unspecified.  The first two end the pipeline at prequantization: when
 * either is set, the escape-cap bit is not.  Returns FZ_OK once the work is enqueued. */
int fz_compress(const float *d_in, const fz_dims *dims, double eb, int eb_mode, void *d_out, void *stream);

/* Timing points of one compression, for callers that measure kernel time
 * (Sec. 4.4 reports kernel time over the input bytes).  Each member is an
 * optional hipEvent_t (as void*, NULL to skip) that fz_compress_timed
 * records on `stream`: range_begin before the value-range pass (REL mode;
 * after the header is initialised), main_begin right before the main
 * compression kernel (which also places the chunks and settles the status
 * word), main_end right after it, done after the last kernel (the same point
 * for the per-field pipeline).  Events bracket launches, so an interval
 * includes the launch gaps inside it. */
typedef struct {
    void *range_begin, *main_begin, *main_end, *done;
} fz_timing;

/* fz_compress_timed -- fz_compress, recording the events of *timing (which
 * may be NULL: then exactly fz_compress).  Same arguments, errors and
 * result. */
int fz_compress_timed(const float *d_in, const fz_dims *dims, double eb, int eb_mode, void *d_out, void *stream,
                      const fz_timing *timing);

/* fz_compress_noalloc -- fz_compress for callers that cannot allocate device
 * memory (work under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same stream, byte for byte, with the compression's
 * scratch (chunk tickets and sizes, partial value ranges, staging slots) in a
 * device array that the library holds, FZ_NOALLOC_SCRATCH_BYTES on each
 * device it runs on, until the process ends.  The call allocates nothing.
 *   d_out     : device buffer of out_bytes >= fz_stream_bound(dims) bytes
 *               (256-byte aligned); on completion it holds the stream
 * The other arguments and the statuses are those of fz_compress.  A field
 * whose scratch does not fit the array (more than about 1.3 million chunks,
 * i.e. about 4.3e10 values) and a d_out smaller than the stream bound return
 * FZ_ERR_ARG at once.  All calls on one device share its array, and each
 * call clears what it needs with a kernel on its own stream: calls that
 * overlap on one device (on different streams, or from several threads)
 * race and must be serialized by the caller. */
#define FZ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fz_compress_noalloc(const float *d_in, const fz_dims *dims, double eb, int eb_mode, void *d_out,
                        size_t out_bytes, void *stream);

/* fz_decompress -- the inverse pipeline (Sec. 4.4 describes it as symmetric
 * to compression).
 *   d_stream     : device pointer to a stream made by fz_compress
 *   stream_bytes : bytes readable at d_stream (at least the stream's size);
 *                  no byte at or past it is ever read.  Below the header,
 *                  table and flags of `dims` (fz_header_bytes): FZ_ERR_ARG
 *   d_out        : N fp32 values (device, written)
 *   dims         : must equal the dims the stream was made with
 *   d_err        : optional device u32; receives 0 or an fz_status code
 *                  (FZ_ERR_STREAM, FZ_ERR_VERSION, FZ_ERR_STATUS) if the
 *                  stream is rejected on the device: bad magic, version,
 *                  status or dims, a total size past stream_bytes, a chunk
 *                  table whose offsets do not follow from the flags'
 *                  popcounts and escape counts, or escape pairs that do not
 *                  match the escape codes.  A chunk found bad is not
 *                  written; a header found bad leaves d_out untouched.
 * Returns FZ_OK once the work is enqueued. */
int fz_decompress(const void *d_stream, size_t stream_bytes, float *d_out, const fz_dims *dims, uint32_t *d_err,
                  void *stream);

/* ------------------------------------------------------------ fp64 input
 * The same pipeline on fp64 fields (FZ_EB_ABS and FZ_EB_REL): the bound's
 * parameters, the value range (REL) and the prequantization q = rint(x *
 * inv) are taken in double (inv = 1 / (2 eb_abs)), so |x' - x| <= eb_abs up
 * to one double rounding of x * inv and of q * 2eb_abs (the Sec. 2.3
 * inequality); the integers q then go through the same encoder, and the
 * stream differs from an fp32 one in the header only: dtype 1 (byte 12),
 * 2 eb_abs and its reciprocal as doubles at bytes 104 and 112 (their fp32
 * roundings, and the range's, fill the fp32 slots for information).
 *
 * fz_compress_bound_f64: bytes of d_out for fz_compress_f64 -- the fp32
 * bound, then the integers q (4 B per value) and the range pass's partials.
 * fz_compress_f64: d_in holds N fp64 values (device); eb_mode FZ_EB_PWREL or
 * any other value returns FZ_ERR_ARG; in ABS mode a 2 eb below the smallest
 * normal double returns FZ_ERR_EB_RANGE at once.  Data-dependent errors and
 * the stream size as for fz_compress.
 * fz_decompress_f64: d_out receives N fp64 values x' = (double) q * 2eb_abs;
 * stream_bytes and d_err as for fz_decompress (an fp32 stream is FZ_ERR_STREAM here, and an
 * fp64 stream is FZ_ERR_STREAM for fz_decompress).
 * The batch and serving layers take fp32 fields only. */
size_t fz_compress_bound_f64(const fz_dims *dims);
int fz_compress_f64(const double *d_in, const fz_dims *dims, double eb, int eb_mode, void *d_out, void *stream);
int fz_decompress_f64(const void *d_stream, size_t stream_bytes, double *d_out, const fz_dims *dims, uint32_t *d_err,
                      void *stream);

/* ------------------------------------------- field-global Lorenzo predictor
 * The classic Lorenzo predictor over the whole field (Sec. 2.3) instead of
 * inside each chunk: a chunk's border cells are predicted from the
 * neighbouring chunk's values (a neighbour outside the field counts 0).  The
 * deltas are coded per chunk exactly as in the chunk-local stream; header
 * byte 15 is 1.  Reconstructions are the same values as with the chunk-local
 * predictor (every stage after prequantization is lossless); only the ratio
 * and the cost differ.  fp32 input, any eb_mode.
 *
 * fz_compress_bound_global: bytes of d_out for fz_compress_global (the fp32
 * bound plus 4 B per value for the integers the chunk kernel reads).
 * fz_compress_global: as fz_compress, with the same arguments and errors.
 * fz_decompress_global_work_bytes: device scratch fz_decompress_global needs
 * (one u32 carry per chunk-box segment of every line along each axis: about
 * 0.44 N bytes for a 3-D field); 0 on invalid dims.
 * fz_decompress_global: as fz_decompress, plus d_work (that many bytes,
 * device, overwritten, 256-byte aligned).  It writes d_out twice (the chunk kernel's local
 * sums, then the values with every axis's carries), so a rejected stream
 * (*d_err set) leaves d_out unspecified.  fz_decompress and the batch layer
 * reject field-global streams (FZ_ERR_STREAM), and fz_decompress_global
 * rejects chunk-local ones. */
size_t fz_compress_bound_global(const fz_dims *dims);
int fz_compress_global(const float *d_in, const fz_dims *dims, double eb, int eb_mode, void *d_out, void *stream);
size_t fz_decompress_global_work_bytes(const fz_dims *dims);
int fz_decompress_global(const void *d_stream, size_t stream_bytes, float *d_out, const fz_dims *dims,
                         uint32_t *d_err, void *d_work, void *stream);

/* ------------------------------------------------------------ batches
 * Many fields of uneven rank and size in a fixed, small number of launches
 * (one persistent compression launch per rank and row-alignment class, over
 * every chunk of every field of that class; one decompression launch).  The
 * bytes each field gets are exactly those of fz_compress / fz_decompress on
 * that field alone.
 *
 * A plan is made once for a list of jobs (it validates them, allocates its
 * own device tables with hipMalloc and copies them there, synchronously);
 * fz_batch_run then only enqueues kernels on `stream`: no allocation, no copy
 * from the host, no synchronization, so a run can be captured in a hipGraph
 * and replayed.  Buffers named by the jobs must stay valid while runs are
 * pending; a plan is not thread-safe, and two pending runs of one plan must
 * be on the same stream. */
typedef struct {
    const float *d_in;   /* N fp32 values (device) */
    fz_dims dims;
    double eb;
    int32_t eb_mode;     /* FZ_EB_ABS or FZ_EB_REL (FZ_EB_PWREL: FZ_ERR_ARG) */
    int32_t reserved;
    void *d_out;         /* fz_compress_bound(&dims) bytes (device) */
} fz_compress_job;

typedef struct {
    const void *d_stream;  /* a stream made by fz_compress (device) */
    fz_dims dims;          /* the dims it was made with */
    float *d_out;          /* N fp32 values (device) */
    uint32_t *d_err;       /* optional device u32, as for fz_decompress */
    uint64_t stream_bytes; /* bytes readable at d_stream, as for fz_decompress */
} fz_decompress_job;

typedef struct fz_batch fz_batch;

/* Make a plan.  On any invalid job returns that job's argument error
 * (FZ_ERR_ARG, or FZ_ERR_EB_RANGE for an unusable absolute bound) and sets
 * *out = NULL; FZ_ERR_HIP if the device tables cannot be made. */
int fz_batch_create_compress(int n, const fz_compress_job *jobs, fz_batch **out);
int fz_batch_create_decompress(int n, const fz_decompress_job *jobs, fz_batch **out);

/* Enqueue one run of the plan on `stream` (asynchronous). */
int fz_batch_run(fz_batch *b, void *stream);

/* Autotune the plan's launch shapes (workgroups per CU of the persistent
 * compression launch, range-pass blocks per field, placement threads per
 * chunk) by timing each candidate on the plan's own fields; runs the plan
 * several times and synchronizes `stream`.  Outputs are rewritten with the
 * same bytes.  Tune before capturing a run in a graph. */
int fz_batch_tune(fz_batch *b, void *stream);

/* Free the plan's device tables (hipFree synchronizes the device). */
int fz_batch_destroy(fz_batch *b);

/* ------------------------------------------------------------- server
 * A request loop on the current device: compress and decompress requests
 * arrive from any host thread; a worker thread admits them in arrival order
 * against an HBM budget (the device bytes each request holds while admitted)
 * and launches the admitted ones in batches (the batch layer's kernels) on
 * `slots` streams, so requests arriving while others run join the next batch
 * as soon as a slot and budget free up, and batches on different streams
 * overlap on the device.  Each result is exactly that of the per-field call.
 * The caller owns the request buffers (device memory) and must keep them
 * until fz_server_wait returns for that request.  The server allocates its
 * streams, device table areas and pinned staging at creation, nothing per
 * request.  Ordering: the server runs requests on streams of its own; work
 * the caller enqueued before submitting (producing d_in, or still using the
 * memory of d_out) is waited for only through ready_event. */
#define FZ_REQ_COMPRESS 0
#define FZ_REQ_DECOMPRESS 1

typedef struct {
    int32_t kind;        /* FZ_REQ_COMPRESS or FZ_REQ_DECOMPRESS */
    int32_t eb_mode;     /* compress: FZ_EB_ABS or FZ_EB_REL (FZ_EB_PWREL: FZ_ERR_ARG) */
    double eb;           /* compress: the error bound */
    fz_dims dims;
    const void *d_in;    /* compress: N fp32 values; decompress: the stream */
    void *d_out;         /* compress: fz_compress_bound bytes; decompress: N fp32 */
    uint32_t *d_err;     /* decompress: optional error word, as for fz_decompress */
    uint64_t hbm_bytes;  /* device bytes charged against the budget while admitted;
                            0: 4N + fz_compress_bound(dims) (compress) or
                            4N + stream_bytes (decompress) */
    uint64_t stream_bytes; /* decompress: bytes readable at d_in (as for fz_decompress) */
    void *ready_event;   /* optional hipEvent_t recorded by the caller after the work that
                            produces d_in and last uses d_out: the request's kernels wait
                            for it on the device; keep it alive until fz_server_wait */
} fz_request;

typedef struct {
    uint64_t submitted, completed, queued;  /* queued: waiting for budget or a slot */
    uint64_t batches;                       /* batch launches */
    double mean_batch;                      /* requests per batch launch */
    uint64_t admission_waits;               /* requests that waited for the budget */
    uint64_t inflight_max_bytes;            /* high-water mark of admitted bytes */
    uint64_t input_bytes;                   /* uncompressed bytes of completed requests */
    double p50_ms, p99_ms, mean_ms, max_ms; /* submit -> completion, completed requests */
    double wall_s;                          /* first submit -> last completion */
} fz_server_report;

typedef struct fz_server fz_server;

/* hbm_budget > 0; slots in 1..16 (streams); max_batch in 1..4096. */
int fz_server_create(uint64_t hbm_budget, int slots, int max_batch, fz_server **out);
/* Validates the request (argument errors return at once; a request larger
 * than the whole budget is FZ_ERR_ARG) and queues it; *ticket names it. */
int fz_server_submit(fz_server *s, const fz_request *r, uint64_t *ticket);
/* Blocks until the request is done; *status is FZ_OK or FZ_ERR_HIP.
 * Data-dependent results are in the output as for the per-field calls. */
int fz_server_wait(fz_server *s, uint64_t ticket, int *status);
/* *done = 1 once the request is done (then fz_server_wait returns at once). */
int fz_server_poll(fz_server *s, uint64_t ticket, int *done);
int fz_server_stats(fz_server *s, fz_server_report *out);
int fz_server_reset_stats(fz_server *s);
/* Finishes every queued request, then frees the server. */
int fz_server_destroy(fz_server *s);

/* ------------------------------------------------------------ quality
 * Distortion of a reconstruction y against its original x, the second of the
 * evaluation metrics of Sec. 4.2 (PSNR over the value range; the paper's
 * bitrate is 32 / compression ratio and needs no device work).  Each
 * difference is taken in double, (double)x - (double)y, rounded once.
 * Results, written to device memory at d_res:
 *   max_abs_err : max |x - y|
 *   mse         : (sum of (x - y)^2) / n, the sum in double
 *   psnr        : 20 log10(vmax - vmin) - 10 log10(mse) dB; +inf when
 *                 mse == 0, -inf when vmax == vmin and mse > 0
 *   vmin, vmax  : the value range of x
 *   n           : values compared
 *   nonfinite   : positions where x or y is NaN or infinite; when > 0 every
 *                 double field is NaN
 * The sum's rounding order is fixed by n alone, so repeated calls give
 * identical bits. */
typedef struct {
    double max_abs_err;
    double mse;
    double psnr;
    double vmin, vmax;
    uint64_t n;
    uint64_t nonfinite;
} fz_quality_report;

/* Device scratch fz_quality needs (per-block partial results): at most
 * 64 KiB.  0 on invalid dims. */
size_t fz_quality_work_bytes(const fz_dims *dims);

/* fz_quality -- d_x, d_y: N fp32 values each (device, read only); d_res:
 * one fz_quality_report (device, written); d_work: fz_quality_work_bytes(dims)
 * bytes (device).  Same dims limits as fz_compress.  Returns FZ_OK once the
 * work is enqueued. */
int fz_quality(const float *d_x, const float *d_y, const fz_dims *dims, fz_quality_report *d_res, void *d_work,
               void *stream);

/* ----------------------------------------------------------- ablation
 * The kernel split the paper compares in Sec. 4.5, rebuilt to measure the
 * same effects on this device; the compression calls above do not use it.
 * Only 3-D fields whose extents are multiples of the chunk box 16 x 32 x 64
 * (slowest first) are accepted (others: FZ_ERR_ARG), with finite input and
 * |x * inv| < 2^31.  A step is one z-plane of one chunk (2048 codes); steps are
 * numbered chunk by chunk (chunks in row-major order), z-planes in order.
 *
 * fz_abl_pred_quant -- dual-quantization with inv = fp32(1 / (2 eb)):
 * q = rint(x * inv), then the chunk-local Lorenzo difference d (zero outside
 * the chunk), written per value in the field's row-major order to d_codes
 * (N u16):
 *   version 1 (the original scheme, Sec. 2.3): d + 512 when -512 < d < 512,
 *             else 0, and d_outliers (N int32, required) receives d where the
 *             code is 0 and 0 elsewhere;
 *   version 2 (the optimized scheme, Sec. 3.2): the 16-bit sign-magnitude
 *             code of d, 0x8000 when |d| > 32767; d_outliers is unused. */
int fz_abl_pred_quant(int version, const float *d_x, const fz_dims *dims, float inv, uint16_t *d_codes,
                      int32_t *d_outliers, void *stream);

/* fz_abl_bitshuffle -- Sec. 3.3: per step a 4096-byte tile at d_tiles +
 * 1024 * step (u32 words): word b * 64 + p holds bit b of the 32 codes of
 * patch p (bit m = cell m; cell m is row m / 8, column m % 8 of the patch;
 * patch p covers rows 4 * (p % 8) .. + 3 and columns 8 * (p / 8) .. + 7 of the
 * step).  d_tiles: N / 2 u32. */
int fz_abl_bitshuffle(const uint16_t *d_codes, const fz_dims *dims, uint32_t *d_tiles, void *stream);

/* fz_abl_mark -- Sec. 3.4: the flags of the tiles: block beta of a step is
 * words 4 * beta .. 4 * beta + 3 of its tile (plane beta / 16 of 128
 * consecutive codes); bit beta % 64 of u64 word 4 * step + beta / 64 of
 * d_flags is set when the block is nonzero.  d_flags: N / 512 u64. */
int fz_abl_mark(const uint32_t *d_tiles, const fz_dims *dims, uint64_t *d_flags, void *stream);

/* fz_abl_bitshuffle_mark -- the two above fused into one kernel (Sec. 3.3):
 * the same tiles and flags, the flags taken from the words in registers. */
int fz_abl_bitshuffle_mark(const uint16_t *d_codes, const fz_dims *dims, uint32_t *d_tiles, uint64_t *d_flags,
                           void *stream);

/* fz_abl_bitshuffle_ballot, fz_abl_bitshuffle_mark_ballot -- the same tiles
 * (and flags) as fz_abl_bitshuffle and fz_abl_bitshuffle_mark, with the
 * transpose done the way Sec. 3.3 does it: the tile's codes pass through
 * shared memory two to a 32-bit word, and one wave vote per bit gathers that
 * bit over the wave's words (64 lanes: one vote gives the plane word of two
 * patches).  512 votes per step instead of the in-register transpose of the
 * other two; the outputs are identical. */
int fz_abl_bitshuffle_ballot(const uint16_t *d_codes, const fz_dims *dims, uint32_t *d_tiles, void *stream);
int fz_abl_bitshuffle_mark_ballot(const uint16_t *d_codes, const fz_dims *dims, uint32_t *d_tiles,
                                  uint64_t *d_flags, void *stream);

/* fz_abl_encode -- Sec. 3.4: d_offsets (steps + 1 u64) receives the exclusive
 * prefix sum of the per-step nonzero block counts (its last entry the
 * total); d_out (N * 2 bytes) the nonzero 16-byte blocks, step by step in
 * block order (its start also holds the per-tile totals of the scan until
 * the blocks are written). */
int fz_abl_encode(const uint32_t *d_tiles, const uint64_t *d_flags, const fz_dims *dims, uint64_t *d_offsets,
                  void *d_out, void *stream);

/* Parse a host copy of the first n >= 128 bytes of a stream. */
int fz_stream_info(const void *h_header, size_t n, fz_info *out);

/* Human-readable name of an fz_status. */
const char *fz_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* FZ_H */
