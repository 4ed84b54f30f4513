/*
 * fzo.c -- the ORACLE: a plain, slow, sequential CPU implementation of the
 * compressor's hot path (dual-quantization, 16-bit code mapping, bitshuffle,
 * zero-block encoder, and the matching decompressor).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant generator
 * with the HIP path: every constant below is restated from the stream-format
 * definition, not included from it.
 *
 * Paper: Zhang et al., "FZ-GPU: A Fast and High-Ratio Lossy Compressor for
 * Scientific Computing Applications on GPUs" (HPDC'23).
 *   - prequantization and its error bound: Sec. 2.3 (the displayed inequality
 *     |round(d/(2eb))*2eb - d| <= eb) and Fig. "error controlling in SZ";
 *   - Lorenzo prediction on the prequantized integers, chunk by chunk:
 *     Sec. 2.3 (dual-quantization) and Sec. 3.2;
 *   - 16-bit code with the sign in the MSB, no radius shift, no outlier split:
 *     Sec. 3.2;
 *   - bitshuffle (bit n of many codes gathered together): Sec. 3.3;
 *   - zero-block encoder (bit flag per data block, prefix sum of block counts
 *     for offsets, copy of the nonzero blocks): Sec. 3.4;
 *   - value-range-relative error bound: Sec. 4.1 ("Baselines");
 *   - point-wise relative error bound through a logarithmic transform of the
 *     data, compressed with the absolute bound that the relative bound
 *     implies: Sec. 4.1 ("Datasets", the HACC treatment);
 *   - decompression is the symmetric inverse: Sec. 4.4.
 * The paper leaves the chunk shape, the order of codes inside a tile, the
 * handling of codes that do not fit in 16 bits, and the stream layout open;
 * this file follows the readings fixed in the stream format v1 (see the
 * comments at each step).
 *
 * Arithmetic: prequantization is fp32 (multiply by the stored reciprocal, then
 * round-half-even), the Lorenzo predictor and its inverse are 32-bit wrapping
 * integer arithmetic, dequantization is one fp32 multiply.  Build with
 * -ffp-contract=off and without fast-math.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "fzo.h"

/* ---------------------------------------------------------------- format v1
 * Restated here (not shared with the HIP path).
 *   chunk box (slowest-first): 3D 16 x 32 x 64, 2D 32 x 1024, 1D 32768
 *   a chunk holds up to 16 "steps" of 2048 codes = 64 patches of 32 codes;
 *   4 consecutive steps form a "layer"; a brick is one bit plane of one patch
 *   over the 4 steps of a layer (128 bits = 16 bytes = one data block).    */
#define FZO_MAGIC 0x314D5A46u /* "FZM1" little-endian */
#define FZO_VERSION 1
#define FZO_HEADER_BYTES 128
#define FZO_STEPS 16
#define FZO_STEP_CODES 2048
#define FZO_PATCHES 64
#define FZO_PATCH_CODES 32
#define FZO_LAYERS 4
#define FZO_CHUNK_CODES (FZO_STEPS * FZO_STEP_CODES)
#define FZO_PLANES 16
#define FZO_FLAG_BYTES_PER_CHUNK (FZO_LAYERS * FZO_PLANES * 8)
/* escapes a chunk may store: 1/32 of its 32768 codes.  A format rule: the
 * worst-case payload of a chunk (every brick nonzero plus this many pairs)
 * sizes the stream bound; where they fall inside the chunk is free.       */
#define FZO_OUTLIER_CAP 1024
#define FZO_ESCAPE 0x8000u

typedef struct {
    int rank;
    int64_t n[3];    /* slowest-first extents, unused trailing dims = 1 */
    int64_t box[3];  /* chunk box, same order */
    int64_t grid[3]; /* chunks per dimension */
    int64_t n_chunks;
    int global; /* Lorenzo predictor over the whole field (1) or inside each chunk (0) */
} geom_t;

static int make_geom(int rank, const int64_t *dims, geom_t *g)
{
    if (rank < 1 || rank > 3 || !dims) return -1;
    memset(g, 0, sizeof(*g));
    g->rank = rank;
    for (int i = 0; i < 3; i++) { g->n[i] = 1; g->box[i] = 1; }
    for (int i = 0; i < rank; i++) {
        if (dims[i] <= 0) return -1;
        g->n[i] = dims[i];
    }
    if (rank == 3) { g->box[0] = 16; g->box[1] = 32; g->box[2] = 64; }
    if (rank == 2) { g->box[0] = 32; g->box[1] = 1024; }
    if (rank == 1) { g->box[0] = 32768; }
    g->n_chunks = 1;
    for (int i = 0; i < 3; i++) {
        g->grid[i] = (g->n[i] + g->box[i] - 1) / g->box[i];
        g->n_chunks *= g->grid[i];
    }
    return 0;
}

/* Map the code index (step s, patch p, cell m) of a chunk to box-relative
 * coordinates (slowest-first).  This is the format's code order.
 *   3D: step = z plane (32 x 64) tiled by 4x8 patches, patches y-fastest;
 *   2D: step = 2 rows x 1024, one 2x16 patch per patch index along x;
 *   1D: step = 2048 consecutive values, 32 per patch.                     */
static void code_to_cell(int rank, int s, int p, int m, int64_t c[3])
{
    c[0] = c[1] = c[2] = 0;
    if (rank == 3) {
        c[0] = s;
        c[1] = 4 * (p % 8) + m / 8;
        c[2] = 8 * (p / 8) + m % 8;
    } else if (rank == 2) {
        c[0] = 2 * s + m / 16;
        c[1] = 16 * p + m % 16;
    } else {
        c[0] = (int64_t)FZO_STEP_CODES * s + FZO_PATCH_CODES * p + m;
    }
}

/* number of stored layers of chunk whose extent along the step dimension is e */
static int layers_of(int rank, int64_t e)
{
    int64_t rows_per_layer = rank == 3 ? 4 : rank == 2 ? 8 : 8192;
    return (int)((e + rows_per_layer - 1) / rows_per_layer);
}

static void chunk_origin(const geom_t *g, int64_t c, int64_t o[3], int64_t ext[3])
{
    int64_t ci[3];
    ci[2] = c % g->grid[2];
    ci[1] = (c / g->grid[2]) % g->grid[1];
    ci[0] = c / (g->grid[2] * g->grid[1]);
    for (int i = 0; i < 3; i++) {
        o[i] = ci[i] * g->box[i];
        ext[i] = g->n[i] - o[i];
        if (ext[i] > g->box[i]) ext[i] = g->box[i];
    }
}

static int64_t lin(const geom_t *g, int64_t a, int64_t b, int64_t c)
{
    return (a * g->n[1] + b) * g->n[2] + c;
}

static int64_t header_bytes(const geom_t *g)
{
    int64_t table = 8 * g->n_chunks;
    table = (table + 15) / 16 * 16;
    return FZO_HEADER_BYTES + table + (int64_t)FZO_FLAG_BYTES_PER_CHUNK * g->n_chunks;
}

int64_t fzo_bound(int rank, const int64_t *dims)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return -1;
    /* every brick nonzero plus the outlier cap, per chunk */
    int64_t per_chunk = (int64_t)FZO_LAYERS * FZO_PLANES * FZO_PATCHES * 16 + FZO_OUTLIER_CAP * 8;
    return header_bytes(&g) + g.n_chunks * per_chunk;
}

/* ------------------------------------------------------------ O1: eb params
 * ABS: eb_abs = eb (vmin = vmax = 0 are recorded).  REL (Sec. 4.1: error bound relative to the value
 * range): eb_abs = eb * (vmax - vmin) in double; a constant field uses
 * eb * |vmax| (or eb if that is 0).  Then ebx2 = fp32(2 eb_abs) and
 * inv = fp32(1 / (double)ebx2); both are stored in the stream and never
 * recomputed by a consumer.                                              */
int fzo_eb_params(const float *x, int64_t n, double eb, int eb_mode,
                  float *ebx2, float *inv, float *vmin, float *vmax)
{
    if (eb_mode == FZO_EB_PWREL) {
        /* PWREL: the step S = floor(eb * 2^24 / (1 + eb)) of the transformed
         * values (see O2b), recorded as an exact float in the ebx2 slot; inv
         * is 0.  Valid for 2 <= S < 2^24. */
        double sd = floor(eb * 16777216.0 / (1.0 + eb));
        *vmin = 0.0f; *vmax = 0.0f; *inv = 0.0f;
        *ebx2 = (sd >= 2.0 && sd < 16777216.0) ? (float)sd : 0.0f;
        return (sd >= 2.0 && sd < 16777216.0) ? 0 : FZO_ERR_EB_RANGE;
    }
    float lo = 0.0f, hi = 0.0f;
    int status = 0;
    if (n > 0 && eb_mode == FZO_EB_REL) { lo = x[0] == 0.0f ? 0.0f : x[0]; hi = lo; }
    /* the value range is only needed (and only recorded) in REL mode */
    for (int64_t i = 0; i < (eb_mode == FZO_EB_REL ? n : 0); i++) {
        if (!isfinite(x[i])) { status |= FZO_ERR_NONFINITE; continue; }
        float v = x[i] == 0.0f ? 0.0f : x[i]; /* -0 counts as +0 */
        if (!isfinite(lo) || v < lo) lo = v;
        if (!isfinite(hi) || v > hi) hi = v;
    }
    *vmin = lo; *vmax = hi;
    double eb_abs = eb;
    if (eb_mode == FZO_EB_REL) {
        if (status) { *ebx2 = 0.0f; *inv = 0.0f; return status; }
        double range = (double)hi - (double)lo;
        if (range > 0.0) eb_abs = eb * range;
        else {
            double a = fabs((double)hi);
            eb_abs = eb * (a > 0.0 ? a : 1.0);
        }
    }
    float e2 = (float)(2.0 * eb_abs);
    float iv = (float)(1.0 / (double)e2);
    *ebx2 = e2; *inv = iv;
    if (!(e2 >= FLT_MIN) || !isfinite(e2) || !isfinite(iv) || !(iv > 0.0f)) status |= FZO_ERR_EB_RANGE;
    return status;
}

/* ---------------------------------------------------- O2: prequantization
 * q = (int32) rintf(x * inv): one fp32 multiply, round half to even.  The
 * product must be finite with |x*inv| < 2^31 so that q fits in int32.    */
int fzo_prequant(const float *x, int64_t n, float inv, int32_t *q)
{
    int status = 0;
    for (int64_t i = 0; i < n; i++) {
        float v = x[i];
        if (!isfinite(v)) { status |= FZO_ERR_NONFINITE; q[i] = 0; continue; }
        float p = v * inv;
        if (!(fabsf(p) < 2147483648.0f)) { status |= FZO_ERR_EB_RANGE; q[i] = 0; continue; }
        q[i] = (int32_t)rintf(p);
    }
    return status;
}

/* ---------------------------------- O2b: the point-wise relative mode
 * The logarithmic transform is the float's own bit pattern: for a finite x,
 * T(x) = b with b = the 31 low bits of x (exponent and mantissa) and the sign
 * of x, which is 2^23 (log2|x| + 127) at every power of two and linear in
 * between.  Quantizing T with the absolute step S changes b by at most S / 2.
 * Within a binade that changes x by a factor of at most 1 + S / 2^24; a change
 * that crosses into the next binade up (where the slope doubles) by at most
 * (S / 2^24) / (1 - S / 2^25).  S = floor(eps * 2^24 / (1 + eps)) gives
 * S / 2^24 <= eps / (1 + eps), which keeps both within 1 + eps / (1 + eps / 2)
 * <= 1 + eps, so |x' - x| <= eps * |x| for normal x; for denormal x
 * (linear bits, no exponent) the change is at most S / 2 units of 2^-149,
 * below eps * 2^-126.
 *   q = sign(x) * floor((b + floor(S / 2)) / S)
 *   x' = the float with the sign of q and the bits min(|q| * S, 0x7F7FFFFF).
 * Zeros of either sign give q = 0 and x' = +0; NaN and infinities are
 * non-finite input.                                                      */
int fzo_prequant_pw(const float *x, int64_t n, uint32_t step, int32_t *q)
{
    int status = 0;
    for (int64_t i = 0; i < n; i++) {
        float v = x[i];
        if (!isfinite(v)) { status |= FZO_ERR_NONFINITE; q[i] = 0; continue; }
        uint32_t bits;
        memcpy(&bits, &v, 4);
        uint32_t b = bits & 0x7FFFFFFFu;
        uint32_t a = (b + step / 2u) / step;
        q[i] = (bits >> 31) ? -(int32_t)a : (int32_t)a;
    }
    return status;
}

float fzo_dequant_pw(int32_t q, uint32_t step)
{
    uint64_t a = q < 0 ? (uint64_t)(-(int64_t)q) : (uint64_t)q;
    uint64_t m = a * (uint64_t)step;
    if (m > 0x7F7FFFFFu) m = 0x7F7FFFFFu;
    uint32_t bits = (uint32_t)m | (q < 0 ? 0x80000000u : 0u);
    float v;
    memcpy(&v, &bits, 4);
    return v;
}

/* ------------------------------------------- O3: chunk-local Lorenzo on q
 * delta = (Dx Dy Dz) q inside the chunk box; a neighbour outside the box is
 * a zero ghost.  Wrapping 32-bit arithmetic.                              */
static uint32_t qat(const geom_t *g, const int32_t *q, const int64_t o[3], int64_t a, int64_t b, int64_t c)
{
    /* a, b, c are box-relative; a ghost is a neighbour before the chunk's
     * origin (chunk-local predictor) or before the field's (O3g) */
    if (g->global) {
        if (o[0] + a < 0 || o[1] + b < 0 || o[2] + c < 0) return 0u;
    } else if (a < 0 || b < 0 || c < 0) {
        return 0u;
    }
    return (uint32_t)q[lin(g, o[0] + a, o[1] + b, o[2] + c)];
}

static int32_t lorenzo_at(const geom_t *g, const int32_t *q, const int64_t o[3], const int64_t r[3])
{
    int64_t a = r[0], b = r[1], c = r[2];
    uint32_t d;
    if (g->rank == 3) {
        d = qat(g, q, o, a, b, c) - qat(g, q, o, a, b, c - 1) - qat(g, q, o, a, b - 1, c)
          - qat(g, q, o, a - 1, b, c) + qat(g, q, o, a, b - 1, c - 1) + qat(g, q, o, a - 1, b, c - 1)
          + qat(g, q, o, a - 1, b - 1, c) - qat(g, q, o, a - 1, b - 1, c - 1);
    } else if (g->rank == 2) {
        /* rank 2: index 0 = y, index 1 = x */
        d = qat(g, q, o, a, b, 0) - qat(g, q, o, a, b - 1, 0) - qat(g, q, o, a - 1, b, 0)
          + qat(g, q, o, a - 1, b - 1, 0);
    } else {
        d = qat(g, q, o, a, 0, 0) - qat(g, q, o, a - 1, 0, 0);
    }
    return (int32_t)d;
}

/* --------------------------------------------------- O4: 16-bit code map
 * Sign in the MSB and the magnitude in the low 15 bits (Sec. 3.2).  A delta
 * that does not fit (|delta| > 32767) is stored as the escape code 0x8000
 * (the otherwise unused "negative zero") plus an outlier pair.            */
int fzo_code_of(int32_t d, uint16_t *code)
{
    if (d == INT32_MIN || d > 32767 || d < -32767) { *code = FZO_ESCAPE; return 1; }
    uint32_t mag = (uint32_t)(d < 0 ? -d : d);
    *code = (uint16_t)((d < 0 ? 0x8000u : 0u) | mag);
    return 0;
}

int32_t fzo_delta_of(uint16_t code)
{
    int32_t mag = code & 0x7fff;
    return (code & 0x8000) ? -mag : mag;
}

/* Codes of one chunk in code-index order (n = s*2048 + p*32 + m), with cells
 * outside the field set to 0.  Returns the number of escapes, which are
 * appended to (oidx, oval) in ascending n.                                */
static int64_t chunk_codes(const geom_t *g, const int32_t *q, int64_t c, uint16_t *codes,
                           uint32_t *oidx, int32_t *oval, int *n_layers)
{
    int64_t o[3], ext[3];
    chunk_origin(g, c, o, ext);
    int L = layers_of(g->rank, ext[0]);
    *n_layers = L;
    int64_t nout = 0;
    for (int64_t n = 0; n < (int64_t)L * 4 * FZO_STEP_CODES; n++) {
        int s = (int)(n / FZO_STEP_CODES), p = (int)((n / FZO_PATCH_CODES) % FZO_PATCHES), m = (int)(n % FZO_PATCH_CODES);
        int64_t r[3];
        code_to_cell(g->rank, s, p, m, r);
        int inside = 1;
        for (int i = 0; i < 3; i++)
            if (r[i] >= ext[i]) inside = 0;
        if (!inside) { codes[n] = 0; continue; }
        int32_t d = lorenzo_at(g, q, o, r);
        if (fzo_code_of(d, &codes[n])) {
            if (nout < FZO_OUTLIER_CAP) { oidx[nout] = (uint32_t)n; oval[nout] = d; }
            nout++;
        }
    }
    return nout;
}

/* ------------------------------------------- O6/O7: bricks and their flags
 * Brick (layer k, plane b, patch p) = 128-bit little-endian integer whose
 * bit 32*t + m is bit b of the code at step 4k+t, patch p, cell m.  It is a
 * data block of Sec. 3.4; its flag is 1 iff it is nonzero.                 */
static void make_brick(const uint16_t *codes, int k, int b, int p, uint32_t w[4])
{
    for (int t = 0; t < 4; t++) {
        uint32_t word = 0;
        for (int m = 0; m < 32; m++) {
            uint16_t code = codes[(int64_t)(4 * k + t) * FZO_STEP_CODES + p * FZO_PATCH_CODES + m];
            word |= (uint32_t)((code >> b) & 1u) << m;
        }
        w[t] = word;
    }
}

static void put32(uint8_t *d, uint32_t v) { for (int i = 0; i < 4; i++) d[i] = (uint8_t)(v >> (8 * i)); }
static void put64(uint8_t *d, uint64_t v) { for (int i = 0; i < 8; i++) d[i] = (uint8_t)(v >> (8 * i)); }
static void put16(uint8_t *d, uint16_t v) { d[0] = (uint8_t)v; d[1] = (uint8_t)(v >> 8); }
static uint32_t get32(const uint8_t *d) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)d[i] << (8 * i); return v; }
static uint64_t get64(const uint8_t *d) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)d[i] << (8 * i); return v; }
static uint16_t get16(const uint8_t *d) { return (uint16_t)(d[0] | (d[1] << 8)); }

typedef struct {
    uint64_t flags[FZO_LAYERS][FZO_PLANES];
    uint32_t *bricks; /* nnz * 4 words */
    int64_t nnz;
    int64_t nout;
    uint32_t *oidx;
    int32_t *oval;
} chunk_out_t;

static void encode_chunk(const geom_t *g, const int32_t *q, int64_t c, chunk_out_t *co)
{
    uint16_t *codes = (uint16_t *)calloc(FZO_CHUNK_CODES, sizeof(uint16_t));
    int L = 0;
    co->oidx = (uint32_t *)malloc(FZO_OUTLIER_CAP * sizeof(uint32_t));
    co->oval = (int32_t *)malloc(FZO_OUTLIER_CAP * sizeof(int32_t));
    co->nout = chunk_codes(g, q, c, codes, co->oidx, co->oval, &L);
    co->bricks = (uint32_t *)malloc((size_t)FZO_LAYERS * FZO_PLANES * FZO_PATCHES * 4 * sizeof(uint32_t));
    co->nnz = 0;
    memset(co->flags, 0, sizeof(co->flags));
    for (int k = 0; k < L; k++)
        for (int b = 0; b < FZO_PLANES; b++)
            for (int p = 0; p < FZO_PATCHES; p++) {
                uint32_t w[4];
                make_brick(codes, k, b, p, w);
                if (w[0] | w[1] | w[2] | w[3]) {
                    co->flags[k][b] |= 1ull << p;
                    memcpy(co->bricks + 4 * co->nnz, w, sizeof(w));
                    co->nnz++;
                }
            }
    free(codes);
}

/* ------------------------------------------------------- O8: the stream
 * header | chunk table {u32 payload offset in 16-B units, u32 outliers} |
 * flags (512 B per chunk) | payload.  Chunk offsets are the exclusive
 * prefix sum of units_c = nnz_c + ceil(out_c / 2) (Sec. 3.4 computes block
 * offsets with a prefix sum).                                             */
/* the header fields that depend on the input type and the bound */
typedef struct {
    int dtype, eb_mode, predictor;
    double eb;
    float ebx2, inv, vmin, vmax;
    double ebx2_64, inv_64; /* fp64 input only (bytes 104 and 112; 0 otherwise) */
} hdr_t;

static int64_t emit_stream(const geom_t *g0, int32_t *q, uint32_t status, const hdr_t *h, uint8_t *out,
                           int64_t cap, uint32_t *status_out, int threads);

int64_t fzo_compress(const float *x, int rank, const int64_t *dims, double eb, int eb_mode,
                     uint8_t *out, int64_t cap, uint32_t *status_out, int threads)
{
    return fzo_compress_pred(x, rank, dims, eb, eb_mode, 0, out, cap, status_out, threads);
}

/* O3g: the field-global Lorenzo predictor (the classic form, Sec. 2.3): the
 * same difference operator over the whole field, a neighbour outside the
 * field being a zero ghost, so that chunk borders are predicted from the
 * neighbouring chunk's values.  The deltas are then coded per chunk exactly
 * as in the chunk-local stream; header byte 15 records the predictor.     */
int64_t fzo_compress_pred(const float *x, int rank, const int64_t *dims, double eb, int eb_mode, int global,
                          uint8_t *out, int64_t cap, uint32_t *status_out, int threads)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return -1;
    if (global != 0 && global != 1) return -1;
    g.global = global;
    if (!(eb > 0.0) || !isfinite(eb) || (eb_mode != FZO_EB_ABS && eb_mode != FZO_EB_REL && eb_mode != FZO_EB_PWREL))
        return -1;
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    if (cap < header_bytes(&g)) return -1;

    hdr_t h;
    memset(&h, 0, sizeof(h));
    h.dtype = 0;
    h.eb_mode = eb_mode;
    h.eb = eb;
    h.predictor = global;
    uint32_t status = (uint32_t)fzo_eb_params(x, N, eb, eb_mode, &h.ebx2, &h.inv, &h.vmin, &h.vmax);
    int32_t *q = (int32_t *)calloc((size_t)N, sizeof(int32_t));
    if (!status)
        status |= (uint32_t)(eb_mode == FZO_EB_PWREL ? fzo_prequant_pw(x, N, (uint32_t)h.ebx2, q)
                                                     : fzo_prequant(x, N, h.inv, q));
    int64_t r = emit_stream(&g, q, status, &h, out, cap, status_out, threads);
    free(q);
    return r;
}

/* ------------------------------------------------ O1d/O2d: fp64 input
 * The same quantizer in double precision (the method is stated for real
 * values; fp64 is the input type of the HACC-like workloads, Sec. 4.1).
 * ABS: eb_abs = eb; REL: eb_abs = eb * (vmax - vmin) over the double values
 * (-0 counts as +0; a constant field uses eb * |vmax|, or eb if that is 0).
 * ebx2 = 2 eb_abs and inv = 1 / ebx2 in double; valid when ebx2 is a normal
 * double and inv is finite.  q = (int32) rint(x * inv) with one double
 * multiply and round-half-even, for finite x with |x * inv| < 2^31;
 * x' = (double) q * ebx2.  Both doubles are recorded in the header (bytes
 * 104 and 112); the fp32 slots hold their fp32 roundings for information. */
int fzo_eb_params_f64(const double *x, int64_t n, double eb, int eb_mode, double *ebx2, double *inv,
                      double *vmin, double *vmax)
{
    double lo = 0.0, hi = 0.0;
    int status = 0, seen = 0;
    *ebx2 = 0.0; *inv = 0.0;
    for (int64_t i = 0; i < (eb_mode == FZO_EB_REL ? n : 0); i++) {
        if (!isfinite(x[i])) { status |= FZO_ERR_NONFINITE; continue; }
        double v = x[i] == 0.0 ? 0.0 : x[i];
        if (!seen || v < lo) lo = v;
        if (!seen || v > hi) hi = v;
        seen = 1;
    }
    *vmin = lo; *vmax = hi;
    if (status) return status;
    double eb_abs = eb;
    if (eb_mode == FZO_EB_REL) {
        double range = hi - lo;
        if (range > 0.0) eb_abs = eb * range;
        else eb_abs = eb * (fabs(hi) > 0.0 ? fabs(hi) : 1.0);
    }
    double e2 = 2.0 * eb_abs, iv = 1.0 / e2;
    if (!(e2 >= DBL_MIN) || !isfinite(e2) || !isfinite(iv) || !(iv > 0.0)) return FZO_ERR_EB_RANGE;
    *ebx2 = e2; *inv = iv;
    return 0;
}

int fzo_prequant_f64(const double *x, int64_t n, double inv, int32_t *q)
{
    int status = 0;
    for (int64_t i = 0; i < n; i++) {
        double v = x[i];
        if (!isfinite(v)) { status |= FZO_ERR_NONFINITE; q[i] = 0; continue; }
        double p = v * inv;
        if (!(fabs(p) < 2147483648.0)) { status |= FZO_ERR_EB_RANGE; q[i] = 0; continue; }
        q[i] = (int32_t)rint(p);
    }
    return status;
}

int64_t fzo_compress_f64(const double *x, int rank, const int64_t *dims, double eb, int eb_mode,
                         uint8_t *out, int64_t cap, uint32_t *status_out, int threads)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return -1;
    if (!(eb > 0.0) || !isfinite(eb) || (eb_mode != FZO_EB_ABS && eb_mode != FZO_EB_REL)) return -1;
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    if (cap < header_bytes(&g)) return -1;

    hdr_t h;
    memset(&h, 0, sizeof(h));
    h.dtype = 1;
    h.eb_mode = eb_mode;
    h.eb = eb;
    double lo, hi;
    uint32_t status = (uint32_t)fzo_eb_params_f64(x, N, eb, eb_mode, &h.ebx2_64, &h.inv_64, &lo, &hi);
    h.ebx2 = (float)h.ebx2_64;
    h.inv = (float)h.inv_64;
    h.vmin = (float)lo;
    h.vmax = (float)hi;
    int32_t *q = (int32_t *)calloc((size_t)N, sizeof(int32_t));
    if (!status) status |= (uint32_t)fzo_prequant_f64(x, N, h.inv_64, q);
    int64_t r = emit_stream(&g, q, status, &h, out, cap, status_out, threads);
    free(q);
    return r;
}

/* O4-O8 and the header: encode the chunks of q (unless status is set) and
 * write the stream. */
static int64_t emit_stream(const geom_t *g0, int32_t *q, uint32_t status, const hdr_t *h, uint8_t *out,
                           int64_t cap, uint32_t *status_out, int threads)
{
    const geom_t g = *g0;
    const int rank = g.rank;
    int64_t H = header_bytes(&g);
    chunk_out_t *co = (chunk_out_t *)calloc((size_t)g.n_chunks, sizeof(chunk_out_t));
    if (!status) {
#ifdef _OPENMP
        if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) if (threads != 1)
#endif
        for (int64_t c = 0; c < g.n_chunks; c++) encode_chunk(&g, q, c, &co[c]);
        /* at most FZO_OUTLIER_CAP escapes per chunk */
        for (int64_t c = 0; c < g.n_chunks; c++)
            if (co[c].nout > FZO_OUTLIER_CAP) status |= FZO_ERR_OUTLIER_CAP;
    }
    (void)threads;

    memset(out, 0, (size_t)H);
    int64_t total = H;
    uint64_t nnz_total = 0, nout_total = 0;
    if (!status) {
        int64_t unit = 0; /* exclusive prefix sum of payload units */
        for (int64_t c = 0; c < g.n_chunks; c++) {
            int64_t units = co[c].nnz + (co[c].nout + 1) / 2;
            uint8_t *tab = out + FZO_HEADER_BYTES + 8 * c;
            put32(tab, (uint32_t)unit);
            put32(tab + 4, (uint32_t)co[c].nout);
            uint8_t *fl = out + H - (int64_t)FZO_FLAG_BYTES_PER_CHUNK * g.n_chunks + FZO_FLAG_BYTES_PER_CHUNK * c;
            for (int k = 0; k < FZO_LAYERS; k++)
                for (int b = 0; b < FZO_PLANES; b++) put64(fl + 8 * (k * FZO_PLANES + b), co[c].flags[k][b]);
            if (H + 16 * (unit + units) > cap) { status = 0xffffffffu; break; }
            uint8_t *pl = out + H + 16 * unit;
            for (int64_t i = 0; i < co[c].nnz; i++)
                for (int t = 0; t < 4; t++) put32(pl + 16 * i + 4 * t, co[c].bricks[4 * i + t]);
            uint8_t *op = pl + 16 * co[c].nnz;
            memset(op, 0, (size_t)(16 * ((co[c].nout + 1) / 2)));
            for (int64_t i = 0; i < co[c].nout; i++) {
                put32(op + 8 * i, co[c].oidx[i]);
                put32(op + 8 * i + 4, (uint32_t)co[c].oval[i]);
            }
            unit += units;
            nnz_total += (uint64_t)co[c].nnz;
            nout_total += (uint64_t)co[c].nout;
        }
        total = H + 16 * unit;
    }
    int overflow = status == 0xffffffffu;
    for (int64_t c = 0; c < g.n_chunks; c++) { free(co[c].bricks); free(co[c].oidx); free(co[c].oval); }
    free(co);

    /* header (F1) */
    put32(out + 0, FZO_MAGIC);
    put16(out + 4, FZO_VERSION);
    put16(out + 6, FZO_HEADER_BYTES);
    put32(out + 8, status);
    out[12] = (uint8_t)h->dtype; /* 0 f32, 1 f64 */
    out[13] = (uint8_t)rank;
    out[14] = (uint8_t)h->eb_mode;
    out[15] = (uint8_t)h->predictor; /* 0 chunk-local Lorenzo, 1 field-global */
    for (int i = 0; i < 3; i++) put64(out + 16 + 8 * i, (uint64_t)g.n[i]);
    memcpy(out + 40, &h->eb, 8);
    memcpy(out + 48, &h->ebx2, 4);
    memcpy(out + 52, &h->inv, 4);
    memcpy(out + 56, &h->vmin, 4);
    memcpy(out + 60, &h->vmax, 4);
    for (int i = 0; i < 3; i++) put16(out + 64 + 2 * i, (uint16_t)g.box[i]);
    put32(out + 72, (uint32_t)g.n_chunks);
    put64(out + 80, nnz_total);
    put64(out + 88, nout_total);
    put64(out + 96, (uint64_t)total);
    if (h->dtype == 1) {
        memcpy(out + 104, &h->ebx2_64, 8);
        memcpy(out + 112, &h->inv_64, 8);
    }
    if (status_out) *status_out = status;
    return overflow ? -2 : total;
}

/* ----------------------------------------------------------- decompressor
 * D1 parse/validate, D2-D3 rebuild the codes of each chunk from the flags
 * and bricks, D4 codes -> delta (escapes take the chunk's pairs), D5 the
 * inverse Lorenzo = inclusive prefix sums along x, then y, then z inside the
 * chunk box (mod 2^32), D6 x' = fp32((float)q * ebx2), or in PWREL mode the
 * inverse transform of q * S (O2b).                                       */
static int decompress_any(const uint8_t *s, int64_t size, float *x, double *x64, int rank, const int64_t *dims,
                          int threads);

int fzo_decompress(const uint8_t *s, int64_t size, float *x, int rank, const int64_t *dims)
{
    return decompress_any(s, size, x, NULL, rank, dims, 1);
}

/* the same with the chunks spread over `threads` OpenMP threads (0: the
 * runtime's default); the result does not depend on the thread count */
int fzo_decompress_threads(const uint8_t *s, int64_t size, float *x, int rank, const int64_t *dims, int threads)
{
    return decompress_any(s, size, x, NULL, rank, dims, threads);
}

/* fp64 streams (dtype 1): x' = (double) q * ebx2, ebx2 the double at byte 104 */
int fzo_decompress_f64(const uint8_t *s, int64_t size, double *x, int rank, const int64_t *dims)
{
    return decompress_any(s, size, NULL, x, rank, dims, 1);
}

/* D2-D6 for chunk c: rebuild its codes from the flags and bricks, decode,
 * undo the predictor and write its values (or, field-global, its deltas).
 * Returns 0 or FZO_DERR_STREAM; *units gets the payload units it read.   */
typedef struct {
    const geom_t *g;
    const uint8_t *s, *flags, *payload;
    int64_t payload_units;
    int mode;
    uint32_t step;
    float ebx2;
    double ebx2_64;
    float *x;
    double *x64;
    uint32_t *field;
} dctx_t;

static int decompress_chunk(const dctx_t *D, int64_t c, uint16_t *codes, int32_t *delta, uint32_t *box, int64_t *units);

static int decompress_any(const uint8_t *s, int64_t size, float *x, double *x64, int rank, const int64_t *dims,
                          int threads)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return FZO_DERR_ARG;
    if (size < FZO_HEADER_BYTES) return FZO_DERR_STREAM;
    if (get32(s) != FZO_MAGIC) return FZO_DERR_STREAM;
    if (get16(s + 4) != FZO_VERSION || get16(s + 6) != FZO_HEADER_BYTES) return FZO_DERR_VERSION;
    if (get32(s + 8) != 0) return FZO_DERR_STATUS;
    if (s[12] != (x64 ? 1 : 0) || s[13] != rank || s[15] > 1) return FZO_DERR_STREAM;
    g.global = s[15];
    for (int i = 0; i < 3; i++)
        if ((int64_t)get64(s + 16 + 8 * i) != g.n[i]) return FZO_DERR_STREAM;
    if ((int64_t)get32(s + 72) != g.n_chunks) return FZO_DERR_STREAM;
    int64_t H = header_bytes(&g);
    int64_t total = (int64_t)get64(s + 96);
    if (total > size || total < H) return FZO_DERR_STREAM;
    float ebx2;
    memcpy(&ebx2, s + 48, 4);
    /* the bound mode: 0 ABS, 1 REL (x' = q * ebx2), 2 PWREL (x' from the
     * transformed value q * S, S recorded in the ebx2 slot) */
    int mode = s[14];
    if (mode > FZO_EB_PWREL || (x64 && mode == FZO_EB_PWREL)) return FZO_DERR_STREAM;
    double ebx2_64 = 0.0;
    if (x64) {
        memcpy(&ebx2_64, s + 104, 8);
        if (!(ebx2_64 >= DBL_MIN) || !isfinite(ebx2_64)) return FZO_DERR_STREAM;
    }
    uint32_t step = 0;
    if (mode == FZO_EB_PWREL) {
        if (!(ebx2 >= 2.0f && ebx2 < 16777216.0f) || ebx2 != floorf(ebx2)) return FZO_DERR_STREAM;
        step = (uint32_t)ebx2;
    }
    const uint8_t *flags = s + H - (int64_t)FZO_FLAG_BYTES_PER_CHUNK * g.n_chunks;
    const uint8_t *payload = s + H;
    int64_t payload_units = (total - H) / 16;

    /* field-global predictor: every chunk's deltas go to one field, summed
     * over the whole field once all chunks are read */
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    uint32_t *field = g.global ? (uint32_t *)calloc((size_t)N, sizeof(uint32_t)) : NULL;
    dctx_t D = {&g, s, flags, payload, payload_units, mode, step, ebx2, ebx2_64, x, x64, field};
    int err = 0;
    int64_t units_seen = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel if (threads != 1) reduction(| : err) reduction(+ : units_seen)
#endif
    {
        uint16_t *codes = (uint16_t *)malloc(FZO_CHUNK_CODES * sizeof(uint16_t));
        int32_t *delta = (int32_t *)malloc(FZO_CHUNK_CODES * sizeof(int32_t));
        uint32_t *box = (uint32_t *)malloc(FZO_CHUNK_CODES * sizeof(uint32_t));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t c = 0; c < g.n_chunks; c++) {
            int64_t u = 0;
            err |= decompress_chunk(&D, c, codes, delta, box, &u);
            units_seen += u;
        }
        free(codes); free(delta); free(box);
    }
    if (!err && g.global) {
        /* D5g: inclusive prefix sums of the deltas along the fastest dim,
         * then the middle, then the slowest, over the whole field (mod 2^32);
         * D6 as above */
        const int64_t n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
        for (int64_t a = 0; a < n0; a++)
            for (int64_t b = 0; b < n1; b++)
                for (int64_t cc = 1; cc < n2; cc++) field[(a * n1 + b) * n2 + cc] += field[(a * n1 + b) * n2 + cc - 1];
        for (int64_t a = 0; a < n0; a++)
            for (int64_t b = 1; b < n1; b++)
                for (int64_t cc = 0; cc < n2; cc++) field[(a * n1 + b) * n2 + cc] += field[(a * n1 + b - 1) * n2 + cc];
        for (int64_t a = 1; a < n0; a++)
            for (int64_t b = 0; b < n1; b++)
                for (int64_t cc = 0; cc < n2; cc++) field[(a * n1 + b) * n2 + cc] += field[((a - 1) * n1 + b) * n2 + cc];
        for (int64_t i = 0; i < N; i++) {
            if (x64) x64[i] = (double)(int32_t)field[i] * ebx2_64;
            else x[i] = mode == FZO_EB_PWREL ? fzo_dequant_pw((int32_t)field[i], step) : (float)(int32_t)field[i] * ebx2;
        }
    }
    free(field);
    if (!err && H + 16 * units_seen != total) err = FZO_DERR_STREAM;
    return err;
}

static int decompress_chunk(const dctx_t *D, int64_t c, uint16_t *codes, int32_t *delta, uint32_t *box, int64_t *units)
{
    const geom_t *gp = D->g;
    const geom_t g = *gp;
    const uint8_t *s = D->s, *flags = D->flags, *payload = D->payload;
    const int64_t payload_units = D->payload_units;
    const int mode = D->mode;
    const uint32_t step = D->step;
    const float ebx2 = D->ebx2;
    const double ebx2_64 = D->ebx2_64;
    float *x = D->x;
    double *x64 = D->x64;
    uint32_t *field = D->field;
    *units = 0;
        int64_t o[3], ext[3];
        chunk_origin(&g, c, o, ext);
        int L = layers_of(g.rank, ext[0]);
        uint32_t off = get32(s + FZO_HEADER_BYTES + 8 * c);
        uint32_t nout = get32(s + FZO_HEADER_BYTES + 8 * c + 4);
        if (nout > FZO_OUTLIER_CAP) return FZO_DERR_STREAM;
        /* D2/D3: rebuild codes */
        memset(codes, 0, FZO_CHUNK_CODES * sizeof(uint16_t));
        int64_t cur = off, nnz = 0;
        for (int k = 0; k < FZO_LAYERS; k++)
            for (int b = 0; b < FZO_PLANES; b++) {
                uint64_t f = get64(flags + FZO_FLAG_BYTES_PER_CHUNK * c + 8 * (k * FZO_PLANES + b));
                if (k >= L && f) return FZO_DERR_STREAM;
                for (int p = 0; p < FZO_PATCHES; p++) {
                    if (!((f >> p) & 1u)) continue;
                    if (cur >= payload_units) return FZO_DERR_STREAM;
                    for (int t = 0; t < 4; t++) {
                        uint32_t w = get32(payload + 16 * cur + 4 * t);
                        for (int m = 0; m < 32; m++)
                            if ((w >> m) & 1u)
                                codes[(4 * k + t) * FZO_STEP_CODES + p * FZO_PATCH_CODES + m] |= (uint16_t)(1u << b);
                    }
                    cur++;
                    nnz++;
                }
            }
        /* D4: codes -> delta; escapes take the pairs in order */
        const uint8_t *op = payload + 16 * cur;
        if (cur + ((int64_t)nout + 1) / 2 > payload_units) return FZO_DERR_STREAM;
        int64_t next_out = 0;
        for (int64_t n = 0; n < (int64_t)L * 4 * FZO_STEP_CODES; n++) {
            if (codes[n] == FZO_ESCAPE) {
                if (next_out >= nout || get32(op + 8 * next_out) != (uint32_t)n) return FZO_DERR_STREAM;
                delta[n] = (int32_t)get32(op + 8 * next_out + 4);
                next_out++;
            } else {
                delta[n] = fzo_delta_of(codes[n]);
            }
        }
        if (next_out != nout) return FZO_DERR_STREAM;
        *units = nnz + ((int64_t)nout + 1) / 2;
        /* scatter delta into the (clipped) box, row-major slowest-first */
        int64_t e0 = ext[0], e1 = ext[1], e2 = ext[2];
        for (int64_t n = 0; n < (int64_t)L * 4 * FZO_STEP_CODES; n++) {
            int64_t r[3];
            code_to_cell(g.rank, (int)(n / FZO_STEP_CODES), (int)((n / FZO_PATCH_CODES) % FZO_PATCHES),
                         (int)(n % FZO_PATCH_CODES), r);
            if (r[0] < e0 && r[1] < e1 && r[2] < e2) box[(r[0] * e1 + r[1]) * e2 + r[2]] = (uint32_t)delta[n];
        }
        if (g.global) {
            for (int64_t a = 0; a < e0; a++)
                for (int64_t b = 0; b < e1; b++)
                    for (int64_t cc = 0; cc < e2; cc++)
                        field[lin(&g, o[0] + a, o[1] + b, o[2] + cc)] = box[(a * e1 + b) * e2 + cc];
            return 0;
        }
        /* D5: inclusive prefix sums along the fastest dim, then the middle,
         * then the slowest (only the dims the rank has) */
        for (int64_t a = 0; a < e0; a++)
            for (int64_t b = 0; b < e1; b++)
                for (int64_t cc = 1; cc < e2; cc++) box[(a * e1 + b) * e2 + cc] += box[(a * e1 + b) * e2 + cc - 1];
        for (int64_t a = 0; a < e0; a++)
            for (int64_t b = 1; b < e1; b++)
                for (int64_t cc = 0; cc < e2; cc++) box[(a * e1 + b) * e2 + cc] += box[(a * e1 + b - 1) * e2 + cc];
        for (int64_t a = 1; a < e0; a++)
            for (int64_t b = 0; b < e1; b++)
                for (int64_t cc = 0; cc < e2; cc++) box[(a * e1 + b) * e2 + cc] += box[((a - 1) * e1 + b) * e2 + cc];
        /* D6: dequantize */
        for (int64_t a = 0; a < e0; a++)
            for (int64_t b = 0; b < e1; b++)
                for (int64_t cc = 0; cc < e2; cc++)
                    if (x64) x64[lin(&g, o[0] + a, o[1] + b, o[2] + cc)] = (double)(int32_t)box[(a * e1 + b) * e2 + cc] * ebx2_64;
                    else x[lin(&g, o[0] + a, o[1] + b, o[2] + cc)] =
                        mode == FZO_EB_PWREL ? fzo_dequant_pw((int32_t)box[(a * e1 + b) * e2 + cc], step)
                                             : (float)(int32_t)box[(a * e1 + b) * e2 + cc] * ebx2;
    return 0;
}

/* ------------------------------------------------------ stage dumps (tests)
 * Codes of chunk c in code-index order (length 4 * 2048 * layers), or the
 * chunk-local Lorenzo delta of the whole field in row-major order.        */
int64_t fzo_chunk_codes(const float *x, int rank, const int64_t *dims, float inv, int64_t c, uint16_t *codes_out)
{
    geom_t g;
    if (make_geom(rank, dims, &g) || c < 0 || c >= g.n_chunks) return -1;
    int64_t N = g.n[0] * g.n[1] * g.n[2];
    int32_t *q = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (fzo_prequant(x, N, inv, q)) { free(q); return -2; }
    uint32_t *oidx = (uint32_t *)malloc(FZO_OUTLIER_CAP * sizeof(uint32_t));
    int32_t *oval = (int32_t *)malloc(FZO_OUTLIER_CAP * sizeof(int32_t));
    int L = 0;
    memset(codes_out, 0, FZO_CHUNK_CODES * sizeof(uint16_t));
    chunk_codes(&g, q, c, codes_out, oidx, oval, &L);
    free(q); free(oidx); free(oval);
    return (int64_t)L * 4 * FZO_STEP_CODES;
}

int fzo_lorenzo_field(const int32_t *q, int rank, const int64_t *dims, int32_t *delta)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return -1;
    for (int64_t c = 0; c < g.n_chunks; c++) {
        int64_t o[3], ext[3];
        chunk_origin(&g, c, o, ext);
        for (int64_t a = 0; a < ext[0]; a++)
            for (int64_t b = 0; b < ext[1]; b++)
                for (int64_t cc = 0; cc < ext[2]; cc++) {
                    int64_t r[3] = {a, b, cc};
                    delta[lin(&g, o[0] + a, o[1] + b, o[2] + cc)] = lorenzo_at(&g, q, o, r);
                }
    }
    return 0;
}

int64_t fzo_header_bytes(int rank, const int64_t *dims)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return -1;
    return header_bytes(&g);
}

int64_t fzo_n_chunks(int rank, const int64_t *dims)
{
    geom_t g;
    if (make_geom(rank, dims, &g)) return -1;
    return g.n_chunks;
}
