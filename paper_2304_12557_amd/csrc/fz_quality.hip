// fz_quality.hip -- distortion of a reconstruction against its original
// (the evaluation metrics of Sec. 4.2: PSNR over the value range, plus the
// maximum pointwise error that the error bound of Sec. 2.3 limits).
//
// Two launches: a grid of blocks that each reduce a fixed stride of the
// field to one partial (sum of squared differences, maximum difference,
// value range of x, count of non-finite positions), then one block that
// folds the partials in a fixed order and derives MSE and PSNR in double.
// The grid size depends on n alone, so the rounding order of the sum, and
// with it every result bit, is the same on every call.  HBM-bound: 8 B read
// per element.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fz.h"
#include "fz_format.hpp"

namespace fz {
namespace {

constexpr int kQualThreads = 256;
constexpr int kQualMaxBlocks = 2048;

struct QualPart {
    double sq;         // sum of (x - y)^2
    double maxerr;     // max |x - y|
    float vmin, vmax;  // range of x over the finite positions
    uint32_t nonfinite;
    uint32_t pad;
};
static_assert(sizeof(QualPart) == 32, "partial layout");

int64_t qual_blocks(int64_t n)
{
    int64_t b = (n + 4 * kQualThreads - 1) / (4 * kQualThreads);
    if (b > kQualMaxBlocks) b = kQualMaxBlocks;
    return b < 1 ? 1 : b;
}

struct Acc {
    double sq, maxerr;
    float vmin, vmax;
    uint32_t nonfinite;

    __device__ void take(float a, float b)
    {
        const bool fin = __builtin_isfinite(a) && __builtin_isfinite(b);
        nonfinite += fin ? 0u : 1u;
        const double e = (double)a - (double)b;  // one rounding to double
        const double e2 = e * e;
        sq += fin ? e2 : 0.0;
        maxerr = fin ? fmax(maxerr, fabs(e)) : maxerr;
        vmin = fin ? fminf(vmin, a) : vmin;
        vmax = fin ? fmaxf(vmax, a) : vmax;
    }
    __device__ void merge(const Acc& o)
    {
        sq += o.sq;
        maxerr = fmax(maxerr, o.maxerr);
        vmin = fminf(vmin, o.vmin);
        vmax = fmaxf(vmax, o.vmax);
        nonfinite += o.nonfinite;
    }
};

// the identity of merge
__device__ Acc acc_zero()
{
    Acc a;
    a.sq = 0.0;
    a.maxerr = 0.0;
    a.vmin = __builtin_inff();
    a.vmax = -__builtin_inff();
    a.nonfinite = 0;
    return a;
}

__device__ Acc shfl_xor_acc(const Acc& a, int m)
{
    Acc o;
    o.sq = __shfl_xor(a.sq, m);
    o.maxerr = __shfl_xor(a.maxerr, m);
    o.vmin = __shfl_xor(a.vmin, m);
    o.vmax = __shfl_xor(a.vmax, m);
    o.nonfinite = (uint32_t)__shfl_xor((int)a.nonfinite, m);
    return o;
}

// Reduce the 256 threads' accumulators of a block in a fixed order; the
// result is valid in thread 0.
__device__ Acc block_reduce(Acc a)
{
    __shared__ Acc s[kQualThreads / 64];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) a.merge(shfl_xor_acc(a, m));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s[w] = a;
    __syncthreads();
    Acc r = acc_zero();
    if (threadIdx.x == 0) {
        r = s[0];
        for (int i = 1; i < kQualThreads / 64; i++) r.merge(s[i]);
    }
    return r;
}

// Block b of the grid takes the float4 groups b*256 + t, then every
// gridDim*256-th after it, and the scalar tail the same way.
__global__ __launch_bounds__(kQualThreads) void k_quality_part(const float* __restrict__ x,
                                                               const float* __restrict__ y, int64_t n,
                                                               QualPart* __restrict__ part)
{
    Acc a = acc_zero();
    const int64_t stride = (int64_t)gridDim.x * kQualThreads;
    const int64_t tid = (int64_t)blockIdx.x * kQualThreads + threadIdx.x;
    const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* y4 = reinterpret_cast<const float4*>(y);
    for (int64_t i = tid; i < n4; i += stride) {
        const float4 u = x4[i], v = y4[i];
        a.take(u.x, v.x);
        a.take(u.y, v.y);
        a.take(u.z, v.z);
        a.take(u.w, v.w);
    }
    for (int64_t i = 4 * n4 + tid; i < n; i += stride) a.take(x[i], y[i]);
    const Acc r = block_reduce(a);
    if (threadIdx.x == 0) {
        QualPart p;
        p.sq = r.sq;
        p.maxerr = r.maxerr;
        p.vmin = r.vmin;
        p.vmax = r.vmax;
        p.nonfinite = r.nonfinite;
        p.pad = 0;
        part[blockIdx.x] = p;
    }
}

__global__ __launch_bounds__(kQualThreads) void k_quality_fold(const QualPart* __restrict__ part, int nparts,
                                                               int64_t n, fz_quality_report* __restrict__ out)
{
    Acc a = acc_zero();
    for (int i = threadIdx.x; i < nparts; i += kQualThreads) {
        Acc o;
        o.sq = part[i].sq;
        o.maxerr = part[i].maxerr;
        o.vmin = part[i].vmin;
        o.vmax = part[i].vmax;
        o.nonfinite = part[i].nonfinite;
        a.merge(o);
    }
    const Acc r = block_reduce(a);
    if (threadIdx.x != 0) return;
    fz_quality_report q;
    q.n = (uint64_t)n;
    q.nonfinite = r.nonfinite;
    if (r.nonfinite) {
        const double nan = __builtin_nan("");
        q.max_abs_err = q.mse = q.psnr = q.vmin = q.vmax = nan;
    } else {
        q.max_abs_err = r.maxerr;
        q.mse = r.sq / (double)n;
        q.vmin = r.vmin;
        q.vmax = r.vmax;
        const double range = (double)r.vmax - (double)r.vmin;
        if (q.mse == 0.0) q.psnr = __builtin_inf();
        else if (range == 0.0) q.psnr = -__builtin_inf();
        else q.psnr = 20.0 * log10(range) - 10.0 * log10(q.mse);
    }
    *out = q;
}

}  // namespace
}  // namespace fz

using namespace fz;

extern "C" {

size_t fz_quality_work_bytes(const fz_dims* dims)
{
    Geom g;
    if (!dims || !make_geom((int)dims->rank, dims->n, &g)) return 0;
    return (size_t)qual_blocks(g.n[0] * g.n[1] * g.n[2]) * sizeof(QualPart);
}

int fz_quality(const float* d_x, const float* d_y, const fz_dims* dims, fz_quality_report* d_res, void* d_work,
               void* stream)
{
    Geom g;
    if (!d_x || !d_y || !d_res || !d_work || !dims || !make_geom((int)dims->rank, dims->n, &g)) return FZ_ERR_ARG;
    if (!aligned_to(d_x, 4) || !aligned_to(d_y, 4) || !aligned_to(d_res, 8) || !aligned_to(d_work, 256)) return FZ_ERR_ARG;
    const int64_t n = g.n[0] * g.n[1] * g.n[2];
    const int64_t blocks = qual_blocks(n);
    hipStream_t st = static_cast<hipStream_t>(stream);
    QualPart* part = static_cast<QualPart*>(d_work);
    hipLaunchKernelGGL(k_quality_part, dim3((unsigned)blocks), dim3(kQualThreads), 0, st, d_x, d_y, n, part);
    if (hipGetLastError() != hipSuccess) return FZ_ERR_HIP;
    hipLaunchKernelGGL(k_quality_fold, dim3(1), dim3(kQualThreads), 0, st, part, (int)blocks, n, d_res);
    return hipGetLastError() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

}  // extern "C"
