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
// prefix sums q one axis at a time: along an axis the global sum of a
// segment is its local sum plus the sum of the totals of the segments before
// it, so per axis k_seg_carry scans the segment-end values of every line
// into a carry per segment and k_seg_add adds it (the last axis also
// dequantizes).  Wrapping 32-bit integer arithmetic throughout.
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

// 64-bit integer division is a long software sequence on the GPU: the
// element loops below index with 32-bit integers whenever the field allows
template <typename I>
__device__ __forceinline__ void cell_of(int64_t i, const Geom& g, int64_t (&c)[3])
{
    const I ii = (I)i, n2 = (I)g.n[2], n1 = (I)g.n[1];
    const I r = ii / n2;
    c[2] = (int64_t)(ii - r * n2);
    c[1] = (int64_t)(r % n1);
    c[0] = (int64_t)(r / n1);
}

template <typename I>
__device__ __forceinline__ int64_t plane_before(int64_t c, int box)
{
    return (int64_t)(((I)c / (I)box) * (I)box) - 1;
}

template <int RANK, typename I>
__global__ __launch_bounds__(kGlobalThreads) void k_face(const float* __restrict__ x, uint8_t* __restrict__ out,
                                                         Geom g)
{
    __shared__ uint32_t s_err[kGlobalThreads / 64];
    Scratch* scr = reinterpret_cast<Scratch*>(out + g.scratch_off);
    if (scr->pre_status) return;  // set before this launch (REL range pass): uniform
    const Quant z = quant_of(out);
    int32_t* p = reinterpret_cast<int32_t*>(out + g.q_off);
    const int64_t n = g.n[0] * g.n[1] * g.n[2];
    const int64_t stride = (int64_t)gridDim.x * kGlobalThreads;
    uint32_t err = 0;
    for (int64_t i = (int64_t)blockIdx.x * kGlobalThreads + threadIdx.x; i < n; i += stride) {
        int64_t c[3];
        cell_of<I>(i, g, c);
        int64_t lo[3];  // the plane just before the chunk along each axis (-1: outside the field)
#pragma unroll
        for (int a = 0; a < 3; a++) lo[a] = a < RANK ? plane_before<I>(c[a], g.box[a]) : -1;
        uint32_t acc = 0;
        uint32_t dummy = 0;
        // subsets of the axes the rank has (axes 0 .. RANK-1; the others
        // have extent 1): bit a of m moves axis a
#pragma unroll
        for (int m = 0; m < (1 << RANK); m++) {
            int64_t q[3] = {c[0], c[1], c[2]};
            bool ghost = false;
            int par = 0;
#pragma unroll
            for (int a = 0; a < RANK; a++) {
                if ((m >> a) & 1) {
                    q[a] = lo[a];
                    ghost |= lo[a] < 0;
                    par ^= 1;
                }
            }
            if (ghost) continue;
            const float v = x[(q[0] * g.n[1] + q[1]) * g.n[2] + q[2]];
            // only the cell's own value reports a status; a face value is
            // another cell's own value
            const uint32_t t = (uint32_t)quant_one(v, z, m == 0 ? err : dummy);
            acc = par ? acc - t : acc + t;
        }
        p[i] = (int32_t)acc;
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
    const int64_t n = g.n[0] * g.n[1] * g.n[2];
    int64_t blocks = (n + kGlobalThreads - 1) / kGlobalThreads;
    blocks = blocks < 1 ? 1 : blocks > 8192 ? 8192 : blocks;
    const bool small = n < (1ll << 32);
    switch (g.rank * 2 + (small ? 1 : 0)) {
        case 7: hipLaunchKernelGGL((k_face<3, uint32_t>), dim3((unsigned)blocks), dim3(kGlobalThreads), 0, st, x, out, g); break;
        case 6: hipLaunchKernelGGL((k_face<3, uint64_t>), dim3((unsigned)blocks), dim3(kGlobalThreads), 0, st, x, out, g); break;
        case 5: hipLaunchKernelGGL((k_face<2, uint32_t>), dim3((unsigned)blocks), dim3(kGlobalThreads), 0, st, x, out, g); break;
        case 4: hipLaunchKernelGGL((k_face<2, uint64_t>), dim3((unsigned)blocks), dim3(kGlobalThreads), 0, st, x, out, g); break;
        case 3: hipLaunchKernelGGL((k_face<1, uint32_t>), dim3((unsigned)blocks), dim3(kGlobalThreads), 0, st, x, out, g); break;
        default: hipLaunchKernelGGL((k_face<1, uint64_t>), dim3((unsigned)blocks), dim3(kGlobalThreads), 0, st, x, out, g); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pre_status(out, g, st);
}

// ------------------------------------------------------------ decompression
template <int RANK, bool VEC4>
__global__ __launch_bounds__(64) void k_decompress_int(const uint8_t* __restrict__ s, int32_t* __restrict__ y, Geom g,
                                                       uint32_t* d_err)
{
    __shared__ float tile[kTileFloats];
    decompress_chunk_any<RANK, VEC4>(s, y, g, d_err, blockIdx.x, threadIdx.x, tile);
}

// The field as (A, L, B) around axis `ax` (A = product of the extents before
// it, L its extent, B the product after it); a line is one (a, b) pair and
// its segments are the chunk box's runs along the axis.
struct Lines {
    int64_t A, L, B, seg, nseg;
};

__host__ __device__ inline Lines lines_of(const Geom& g, int ax)
{
    Lines l;
    l.A = 1;
    l.B = 1;
    for (int i = 0; i < ax; i++) l.A *= g.n[i];
    for (int i = ax + 1; i < 3; i++) l.B *= g.n[i];
    l.L = g.n[ax];
    l.seg = g.box[ax];
    l.nseg = (l.L + l.seg - 1) / l.seg;
    return l;
}

// carry[j][line] = sum of the values at the ends of segments 0 .. j-1 of the line
__global__ __launch_bounds__(kGlobalThreads) void k_seg_carry(const uint32_t* __restrict__ f, uint32_t* __restrict__ carry,
                                                              Lines l)
{
    const int64_t nlines = l.A * l.B;
    const int64_t stride = (int64_t)gridDim.x * kGlobalThreads;
    for (int64_t t = (int64_t)blockIdx.x * kGlobalThreads + threadIdx.x; t < nlines; t += stride) {
        const int64_t a = t / l.B, b = t % l.B;
        const uint32_t* line = f + a * l.L * l.B + b;
        uint32_t run = 0;
        for (int64_t j = 0; j < l.nseg; j++) {
            carry[j * nlines + t] = run;
            const int64_t end = (j + 1) * l.seg < l.L ? (j + 1) * l.seg - 1 : l.L - 1;
            run += line[end * l.B];
        }
    }
}

// f += carry of its segment; on the last axis also dequantize (Sec. 2.3; the
// point-wise mode's inverse transform) and store the fp32 value in place
template <bool LAST, typename I>
__global__ __launch_bounds__(kGlobalThreads) void k_seg_add(uint32_t* __restrict__ f, const uint32_t* __restrict__ carry,
                                                            Lines l, const uint8_t* __restrict__ s)
{
    const I B = (I)l.B, L = (I)l.L, seg = (I)l.seg, nlines = (I)(l.A * l.B);
    const int64_t n = l.A * l.L * l.B;
    const int64_t stride = (int64_t)gridDim.x * kGlobalThreads;
    float ebx2 = 0.0f;
    uint32_t step = 0;
    bool pw = false;
    if (LAST) {
        ebx2 = *reinterpret_cast<const float*>(s + kOffEbx2);
        pw = s[kOffEbMode] == 2;
        step = pw ? (uint32_t)ebx2 : 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * kGlobalThreads + threadIdx.x; i < n; i += stride) {
        const I ii = (I)i;
        const I r = ii / B, b = ii - r * B;
        const I a = r / L, k = r - a * L;
        const uint32_t v = f[i] + carry[(int64_t)(k / seg) * (int64_t)nlines + (int64_t)(a * B + b)];
        if (LAST) {
            const int q = (int)v;
            f[i] = __float_as_uint(pw ? pw_dequant(q, step) : (float)q * ebx2);
        } else {
            f[i] = v;
        }
    }
}

// A rejected stream (header or chunk check) sets d_err; the output is then
// unspecified (the carry passes run on whatever the chunk kernel left).
__global__ void k_clear_err_g(uint32_t* p)
{
    if (threadIdx.x == 0) *p = 0u;
}

template <int RANK, bool VEC4>
static hipError_t launch_rank_int(const uint8_t* s, int32_t* y, const Geom& g, uint32_t* d_err, hipStream_t st)
{
    hipLaunchKernelGGL((k_decompress_int<RANK, VEC4>), dim3((unsigned)g.n_chunks), dim3(64), 0, st, s, y, g, d_err);
    return hipGetLastError();
}

size_t global_work_bytes(const Geom& g)
{
    int64_t most = 0;
    for (int ax = 0; ax < g.rank; ax++) {
        const Lines l = lines_of(g, ax);
        const int64_t b = 4 * l.A * l.B * l.nseg;
        most = b > most ? b : most;
    }
    return (size_t)most;
}

hipError_t launch_decompress_global(const uint8_t* s, float* y, const Geom& g, uint32_t* d_err, void* work,
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
        case 7: e = launch_rank_int<3, true>(s, yi, g, d_err, st); break;
        case 6: e = launch_rank_int<3, false>(s, yi, g, d_err, st); break;
        case 5: e = launch_rank_int<2, true>(s, yi, g, d_err, st); break;
        case 4: e = launch_rank_int<2, false>(s, yi, g, d_err, st); break;
        case 3: e = launch_rank_int<1, true>(s, yi, g, d_err, st); break;
        default: e = launch_rank_int<1, false>(s, yi, g, d_err, st); break;
    }
    if (e != hipSuccess) return e;
    uint32_t* f = reinterpret_cast<uint32_t*>(y);
    uint32_t* carry = static_cast<uint32_t*>(work);
    // the contiguous axis first, then the middle, then the slowest: the
    // order of the inclusive sums of the inverse predictor
    for (int ax = g.rank - 1; ax >= 0; ax--) {
        const Lines l = lines_of(g, ax);
        const int64_t nlines = l.A * l.B, n = l.A * l.L * l.B;
        int64_t bc = (nlines + kGlobalThreads - 1) / kGlobalThreads;
        bc = bc < 1 ? 1 : bc > 4096 ? 4096 : bc;
        hipLaunchKernelGGL(k_seg_carry, dim3((unsigned)bc), dim3(kGlobalThreads), 0, st, f, carry, l);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        int64_t ba = (n + kGlobalThreads - 1) / kGlobalThreads;
        ba = ba < 1 ? 1 : ba > 8192 ? 8192 : ba;
        const bool small = n < (1ll << 32);
        if (ax == 0 && small)
            hipLaunchKernelGGL((k_seg_add<true, uint32_t>), dim3((unsigned)ba), dim3(kGlobalThreads), 0, st, f, carry, l, s);
        else if (ax == 0)
            hipLaunchKernelGGL((k_seg_add<true, uint64_t>), dim3((unsigned)ba), dim3(kGlobalThreads), 0, st, f, carry, l, s);
        else if (small)
            hipLaunchKernelGGL((k_seg_add<false, uint32_t>), dim3((unsigned)ba), dim3(kGlobalThreads), 0, st, f, carry, l, s);
        else
            hipLaunchKernelGGL((k_seg_add<false, uint64_t>), dim3((unsigned)ba), dim3(kGlobalThreads), 0, st, f, carry, l, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fz
