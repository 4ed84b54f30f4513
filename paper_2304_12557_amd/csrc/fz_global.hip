// fz_global.hip -- the field-global Lorenzo predictor of libfzmi (gfx950).
//
// The classic Lorenzo predictor runs over the whole field (Sec. 2.3): a
// chunk's border cells are predicted from the neighbouring chunk's values.
// The stream stores the field-global deltas d chunk by chunk, exactly as the
// chunk-local stream stores its own, and header byte 15 says which.
//
// Compression reuses the chunk kernel unchanged.  That kernel takes the
// chunk-local Lorenzo difference of its input, so it is fed the integers p
// whose chunk-local difference is d: the inclusion-exclusion of q over the
// chunk's lower faces, p(c) = sum over subsets S of the axes of (-1)^|S|
// q(c with the axes in S moved to the plane just before the chunk), a
// neighbour outside the field counting 0.  k_face computes p from the input
// (prequantizing the few face values it needs on the fly) into the integer
// buffer behind the fp32 bound.
//
// Decompression runs the chunk kernel with integer output, which yields the
// chunk-local prefix sums p again, and then turns them into the field-global
// prefix sums q: per axis a small kernel computes the carries of every line's
// segments from the segment-end values (k_seg_carry), and one pass adds them
// all and dequantizes (k_seg_final).  Wrapping 32-bit integer arithmetic
// throughout.
#include <hip/hip_runtime.h>

#include "fz.h"
#include "fz_decompress_dev.hpp"
#include "fz_kernels.hpp"

namespace fz {

constexpr int kGlobalThreads = 256;

// one value through the stream's quantizer; err collects NaN/Inf (and in
// the grid modes |x * inv| >= 2^31)
__device__ __forceinline__ int32_t quant_one(float v, const Quant& z, uint32_t& err)
{
    if (!(__builtin_fabsf(v) <= 3.40282347e38f)) {
        err |= kErrNonfinite;
        return 0;
    }
    if (z.step) return pw_quant(v, z);
    const float p = v * z.inv;
    if (!(__builtin_fabsf(p) < 2147483648.0f)) {
        err |= kErrEbRange;
        return 0;
    }
    return (int32_t)__builtin_rintf(p);
}

// launch shape of the row kernels: runs of 256 cells along the contiguous
// axis in x, rows (all other coordinates) in y, both grid-strided
inline dim3 row_grid(const Geom& g)
{
    const int64_t nx = g.n[g.rank - 1], nrows = g.n[0] * g.n[1] * g.n[2] / nx;
    int64_t bx = (nx + kGlobalThreads - 1) / kGlobalThreads, by = nrows;
    bx = bx > (1 << 16) ? (1 << 16) : bx;
    by = by > 65535 ? 65535 : by;
    while (bx * by > (1 << 18) && by > 1) by = (by + 1) / 2;  // a few hundred thousand blocks at most
    return dim3((unsigned)bx, (unsigned)by);
}

// p of one cell from the quantized values q(c) of the cell and of its face
// neighbours: a block takes 256 consecutive cells of one row (every
// coordinate but the contiguous one fixed), so the row's coordinates, the
// planes before the chunk along the slow axes and their row addresses are
// uniform.  Only the cell's own value reports a status; a face value is
// another cell's own value.
template <int RANK>
__global__ __launch_bounds__(kGlobalThreads) void k_face(const float* __restrict__ x, uint8_t* __restrict__ out,
                                                         Geom g)
{
    __shared__ uint32_t s_err[kGlobalThreads / 64];
    Scratch* scr = reinterpret_cast<Scratch*>(out + g.scratch_off);
    if (scr->pre_status) return;  // set before this launch (REL range pass): uniform
    const Quant z = quant_of(out);
    int32_t* p = reinterpret_cast<int32_t*>(out + g.q_off);
    const int64_t nx = g.n[RANK - 1];
    const int64_t nrows = g.n[0] * g.n[1] * g.n[2] / nx;
    // chunk boxes are powers of two: the planes before a chunk come from shifts
    const int shx = __builtin_ctz((unsigned)g.box[RANK - 1]);
    const int sh0 = __builtin_ctz((unsigned)g.box[0]), sh1 = __builtin_ctz((unsigned)g.box[1]);
    uint32_t err = 0, dummy = 0;
    auto qv = [&](int64_t idx, bool own) -> uint32_t { return (uint32_t)quant_one(x[idx], z, own ? err : dummy); };
    // a 2-D grid: rows along y, runs of 256 cells along x (no division per run)
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * kGlobalThreads + threadIdx.x; c < nx; c += (int64_t)gridDim.x * kGlobalThreads) {
        const int64_t X = ((c >> shx) << shx) - 1;  // the column before the chunk (-1: outside the field)
        uint32_t acc;
        if constexpr (RANK == 1) {
            acc = qv(c, true) - (X >= 0 ? qv(X, false) : 0u);
        } else if constexpr (RANK == 2) {
            const int64_t Y = ((row >> sh0) << sh0) - 1;
            const int64_t r0 = row * nx, rY = Y * nx;
            acc = qv(r0 + c, true);
            if (X >= 0) acc -= qv(r0 + X, false);
            if (Y >= 0) {
                acc -= qv(rY + c, false);
                if (X >= 0) acc += qv(rY + X, false);
            }
        } else {
            const int64_t c0 = row / g.n[1], c1 = row - c0 * g.n[1];
            const int64_t Z = ((c0 >> sh0) << sh0) - 1, Y = ((c1 >> sh1) << sh1) - 1;
            const int64_t r00 = row * nx, rZ0 = (Z * g.n[1] + c1) * nx, r0Y = (c0 * g.n[1] + Y) * nx,
                          rZY = (Z * g.n[1] + Y) * nx;
            acc = qv(r00 + c, true);
            if (X >= 0) acc -= qv(r00 + X, false);
            if (Y >= 0) {
                acc -= qv(r0Y + c, false);
                if (X >= 0) acc += qv(r0Y + X, false);
            }
            if (Z >= 0) {
                acc -= qv(rZ0 + c, false);
                if (X >= 0) acc += qv(rZ0 + X, false);
                if (Y >= 0) {
                    acc += qv(rZY + c, false);
                    if (X >= 0) acc -= qv(rZY + X, false);
                }
            }
        }
        p[row * nx + c] = (int32_t)acc;
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) err |= (uint32_t)__shfl_xor((int)err, sh);
    if ((threadIdx.x & 63) == 0) s_err[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kGlobalThreads / 64; i++) err |= s_err[i];
        if (err) {
            atomicOr(reinterpret_cast<uint32_t*>(out + kOffStatus), err);
            *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off;
        }
    }
}

hipError_t launch_face(const float* x, uint8_t* out, const Geom& g, hipStream_t st)
{
    const dim3 grid = row_grid(g);
    switch (g.rank) {
        case 3: hipLaunchKernelGGL(k_face<3>, grid, dim3(kGlobalThreads), 0, st, x, out, g); break;
        case 2: hipLaunchKernelGGL(k_face<2>, grid, dim3(kGlobalThreads), 0, st, x, out, g); break;
        default: hipLaunchKernelGGL(k_face<1>, grid, dim3(kGlobalThreads), 0, st, x, out, g); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pre_status(out, g, st);
}

// ------------------------------------------------------------ decompression
template <int RANK, bool VEC4>
__global__ __launch_bounds__(64, 2) void k_decompress_int(const uint8_t* __restrict__ s, uint64_t sb,
                                                       int32_t* __restrict__ y, Geom g, uint32_t* d_err)
{
    __shared__ float tile[kTileFloats];
    decompress_chunk_any<RANK, VEC4>(s, sb, y, g, d_err, blockIdx.x, threadIdx.x, tile);
}

// Carries of the field-global prefix sums.  Along axis ax the field splits
// into lines (every cell with the other coordinates fixed) and each line into
// segments of the chunk box's extent along ax (a power of two).  After the
// chunk kernel the field holds p, the chunk-local sums.  Taking the axes from
// the contiguous one to the slowest, the global sum along an axis of a value
// that already holds the earlier axes' carries is its local sum plus the
// totals of the line's earlier segments; those totals are the values at the
// segment ends, which are p plus the earlier axes' carries there.  So per axis
// one small kernel reads only the segment ends and writes the carries
// (carry[ax][j][line] = sum over the segments before j), and one final pass
// adds every axis's carry to p and dequantizes.  The sums commute, and all of
// it is wrapping 32-bit arithmetic.
struct Carries {
    int rank;
    int64_t n[3];
    int sh[3];          // log2 of the chunk box along each axis
    int64_t nlines[3];  // lines along each axis
    int64_t nseg[3];    // segments per line
    int64_t off[3];     // start of each axis's carries in the work buffer (u32 units)
};

inline Carries carries_of(const Geom& g)
{
    Carries c;
    c.rank = g.rank;
    int64_t off = 0;
    for (int a = 0; a < 3; a++) {
        c.n[a] = g.n[a];
        c.sh[a] = __builtin_ctz((unsigned)g.box[a]);
        c.nlines[a] = g.n[0] * g.n[1] * g.n[2] / g.n[a];
        c.nseg[a] = (g.n[a] + g.box[a] - 1) / g.box[a];
        c.off[a] = off;
        if (a < g.rank) off += c.nlines[a] * c.nseg[a];
    }
    return c;
}

// the line of axis ax through cell (c0, c1, c2)
__device__ __forceinline__ int64_t line_of(const Carries& k, int ax, int64_t c0, int64_t c1, int64_t c2)
{
    return ax == 2 ? c0 * k.n[1] + c1 : ax == 1 ? c0 * k.n[2] + c2 : c1 * k.n[2] + c2;
}

// the sum of the carries of axes first .. rank-1 at cell (c0, c1, c2)
__device__ __forceinline__ uint32_t carry_sum(const Carries& k, const uint32_t* __restrict__ w, int first, int64_t c0,
                                              int64_t c1, int64_t c2)
{
    uint32_t v = 0;
    const int64_t c[3] = {c0, c1, c2};
    for (int ax = first; ax < k.rank; ax++)
        v += w[k.off[ax] + (c[ax] >> k.sh[ax]) * k.nlines[ax] + line_of(k, ax, c0, c1, c2)];
    return v;
}

__global__ __launch_bounds__(kGlobalThreads) void k_seg_carry(const uint32_t* __restrict__ p, uint32_t* __restrict__ w,
                                                              Carries k, int ax)
{
    const int64_t nl = k.nlines[ax];
    const int64_t stride = (int64_t)gridDim.x * kGlobalThreads;
    for (int64_t t = (int64_t)blockIdx.x * kGlobalThreads + threadIdx.x; t < nl; t += stride) {
        // the other two coordinates of line t
        int64_t c[3];
        if (ax == 2) { c[0] = t / k.n[1]; c[1] = t % k.n[1]; }
        else if (ax == 1) { c[0] = t / k.n[2]; c[2] = t % k.n[2]; }
        else { c[1] = t / k.n[2]; c[2] = t % k.n[2]; }
        uint32_t run = 0;
        for (int64_t j = 0; j < k.nseg[ax]; j++) {
            w[k.off[ax] + j * nl + t] = run;
            const int64_t end = ((j + 1) << k.sh[ax]) < k.n[ax] ? ((j + 1) << k.sh[ax]) - 1 : k.n[ax] - 1;
            c[ax] = end;
            run += p[(c[0] * k.n[1] + c[1]) * k.n[2] + c[2]] + carry_sum(k, w, ax + 1, c[0], c[1], c[2]);
        }
    }
}

// q = p + the carries of every axis, dequantized (Sec. 2.3; the point-wise
// mode's inverse transform) and stored as fp32 in place.  A block takes 256
// consecutive cells of one row (the cells that share every coordinate but
// the contiguous one), so the row's coordinates and carry offsets are
// uniform and no per-cell division is needed.
template <int RANK>
__global__ __launch_bounds__(kGlobalThreads) void k_seg_final(uint32_t* __restrict__ f, const uint32_t* __restrict__ w,
                                                              Carries k, const uint8_t* __restrict__ s)
{
    const float ebx2 = *reinterpret_cast<const float*>(s + kOffEbx2);
    const bool pw = s[kOffEbMode] == 2;
    const uint32_t step = pw ? (uint32_t)ebx2 : 0u;
    const int64_t nx = k.n[RANK - 1];
    const int64_t nrows = k.n[0] * k.n[1] * k.n[2] / nx;
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y)
    for (int64_t x = (int64_t)blockIdx.x * kGlobalThreads + threadIdx.x; x < nx; x += (int64_t)gridDim.x * kGlobalThreads) {
        uint32_t c;
        if constexpr (RANK == 3) {
            const int64_t c0 = row / k.n[1], c1 = row - c0 * k.n[1];
            c = w[k.off[2] + (x >> k.sh[2]) * k.nlines[2] + row] +
                w[k.off[1] + (c1 >> k.sh[1]) * k.nlines[1] + c0 * k.n[2] + x] +
                w[k.off[0] + (c0 >> k.sh[0]) * k.nlines[0] + c1 * k.n[2] + x];
        } else if constexpr (RANK == 2) {
            c = w[k.off[1] + (x >> k.sh[1]) * k.nlines[1] + row] + w[k.off[0] + (row >> k.sh[0]) * k.nlines[0] + x];
        } else {
            c = w[k.off[0] + (x >> k.sh[0])];
        }
        const int64_t i = row * nx + x;
        const int q = (int)(f[i] + c);
        f[i] = __float_as_uint(pw ? pw_dequant(q, step) : (float)q * ebx2);
    }
}

// A rejected stream (header or chunk check) sets d_err; the output is then
// unspecified (the carry passes run on whatever the chunk kernel left).
__global__ void k_clear_err_g(uint32_t* p)
{
    if (threadIdx.x == 0) *p = 0u;
}

template <int RANK, bool VEC4>
static hipError_t launch_rank_int(const uint8_t* s, uint64_t sb, int32_t* y, const Geom& g, uint32_t* d_err,
                                  hipStream_t st)
{
    hipLaunchKernelGGL((k_decompress_int<RANK, VEC4>), dim3((unsigned)g.n_chunks), dim3(64), 0, st, s, sb, y, g, d_err);
    return hipGetLastError();
}

size_t global_work_bytes(const Geom& g)
{
    const Carries k = carries_of(g);
    int64_t total = 0;
    for (int ax = 0; ax < g.rank; ax++) total += k.nlines[ax] * k.nseg[ax];
    return (size_t)(4 * total);
}

hipError_t launch_decompress_global(const uint8_t* s, uint64_t sb, float* y, const Geom& g, uint32_t* d_err, void* work,
                                    hipStream_t st)
{
    hipError_t e;
    if (d_err) {
        hipLaunchKernelGGL(k_clear_err_g, dim3(1), dim3(64), 0, st, d_err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int32_t* yi = reinterpret_cast<int32_t*>(y);
    const bool vec4 = (reinterpret_cast<uintptr_t>(y) & 15) == 0 && (g.rank == 1 || (g.n[g.rank - 1] & 3) == 0);
    switch (g.rank * 2 + (vec4 ? 1 : 0)) {
        case 7: e = launch_rank_int<3, true>(s, sb, yi, g, d_err, st); break;
        case 6: e = launch_rank_int<3, false>(s, sb, yi, g, d_err, st); break;
        case 5: e = launch_rank_int<2, true>(s, sb, yi, g, d_err, st); break;
        case 4: e = launch_rank_int<2, false>(s, sb, yi, g, d_err, st); break;
        case 3: e = launch_rank_int<1, true>(s, sb, yi, g, d_err, st); break;
        default: e = launch_rank_int<1, false>(s, sb, yi, g, d_err, st); break;
    }
    if (e != hipSuccess) return e;
    uint32_t* f = reinterpret_cast<uint32_t*>(y);
    uint32_t* w = static_cast<uint32_t*>(work);
    const Carries k = carries_of(g);
    // the contiguous axis first, then the middle, then the slowest
    for (int ax = g.rank - 1; ax >= 0; ax--) {
        int64_t bc = (k.nlines[ax] + kGlobalThreads - 1) / kGlobalThreads;
        bc = bc < 1 ? 1 : bc > 4096 ? 4096 : bc;
        hipLaunchKernelGGL(k_seg_carry, dim3((unsigned)bc), dim3(kGlobalThreads), 0, st, f, w, k, ax);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const dim3 grid = row_grid(g);
    switch (g.rank) {
        case 3: hipLaunchKernelGGL(k_seg_final<3>, grid, dim3(kGlobalThreads), 0, st, f, w, k, s); break;
        case 2: hipLaunchKernelGGL(k_seg_final<2>, grid, dim3(kGlobalThreads), 0, st, f, w, k, s); break;
        default: hipLaunchKernelGGL(k_seg_final<1>, grid, dim3(kGlobalThreads), 0, st, f, w, k, s); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace fz
