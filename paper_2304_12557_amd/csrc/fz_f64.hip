// fz_f64.hip -- the fp64-input front end and the fp64 decompression kernel
// of libfzmi (gfx950).
//
// fp64 fields are quantized in double precision (Sec. 2.3's quantizer with
// q = rint(x * inv), inv = 1 / (2 eb) as doubles) by a pass of their own,
// which writes the integers q (4 B per value) behind the fp32 bound of the
// output buffer; the compression kernel then reads q in place of fp32 values
// and the rest of the pipeline is unchanged.  REL mode first takes the value
// range in double (Sec. 4.1).  Decompression runs the fp32 kernel's device
// code with an fp64 dequantization and fp64 stores.
#include <hip/hip_runtime.h>

#include "fz.h"
#include "fz_decompress_dev.hpp"
#include "fz_kernels.hpp"

namespace fz {

constexpr int kF64Threads = 256;

__device__ __forceinline__ bool finite64(double v) { return __builtin_fabs(v) <= 1.7976931348623157e308; }

// Partial range of block blk: min and max over the finite values (-0 as +0)
// and a flag for non-finite ones.
__global__ __launch_bounds__(kF64Threads) void k_minmax64(const double* __restrict__ x, int64_t n,
                                                         uint8_t* __restrict__ out, Geom g)
{
    __shared__ double s_lo[kF64Threads / 64], s_hi[kF64Threads / 64];
    __shared__ uint32_t s_bad[kF64Threads / 64];
    double lo = __builtin_inf(), hi = -__builtin_inf();
    uint32_t bad = 0;
    auto take = [&](double v) {
        if (!finite64(v)) {
            bad = 1;
        } else {
            v = v == 0.0 ? 0.0 : v;
            lo = __builtin_fmin(lo, v);
            hi = __builtin_fmax(hi, v);
        }
    };
    const int64_t stride = (int64_t)gridDim.x * kF64Threads;
    const int64_t tid = (int64_t)blockIdx.x * kF64Threads + threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const int64_t n2 = vec ? n / 2 : 0;
    const fz_f64x2* x2 = reinterpret_cast<const fz_f64x2*>(x);
    for (int64_t i = tid; i < n2; i += stride) {
        const fz_f64x2 v = __builtin_nontemporal_load(x2 + i);
        take(v.x);
        take(v.y);
    }
    for (int64_t k = 2 * n2 + tid; k < n; k += stride) take(x[k]);
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
        lo = __builtin_fmin(lo, __shfl_xor(lo, sh));
        hi = __builtin_fmax(hi, __shfl_xor(hi, sh));
        bad |= (uint32_t)__shfl_xor((int)bad, sh);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_lo[w] = lo; s_hi[w] = hi; s_bad[w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kF64Threads / 64; i++) {
            lo = __builtin_fmin(lo, s_lo[i]);
            hi = __builtin_fmax(hi, s_hi[i]);
            bad |= s_bad[i];
        }
        double* part = reinterpret_cast<double*>(out + g.part64_off);
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
        reinterpret_cast<uint32_t*>(out + g.part64_off + 16 * kMinmaxBlocks)[blockIdx.x] = bad;
    }
}

// Fold the partials, derive 2 eb_abs and its reciprocal in double and write
// them (and their fp32 roundings, with the range's) to the header.  A
// non-finite value or an unusable bound ends the pipeline here: the status
// goes to the header and the scratch, the stream to its header size.
__global__ __launch_bounds__(kF64Threads) void k_params64(uint8_t* __restrict__ out, Geom g, double eb, int nparts)
{
    __shared__ double s_lo[kF64Threads / 64], s_hi[kF64Threads / 64];
    __shared__ uint32_t s_bad[kF64Threads / 64];
    const double* part = reinterpret_cast<const double*>(out + g.part64_off);
    const uint32_t* pbad = reinterpret_cast<const uint32_t*>(out + g.part64_off + 16 * kMinmaxBlocks);
    double lo = __builtin_inf(), hi = -__builtin_inf();
    uint32_t bad = 0;
    for (int i = threadIdx.x; i < nparts; i += kF64Threads) {
        lo = __builtin_fmin(lo, part[2 * i]);
        hi = __builtin_fmax(hi, part[2 * i + 1]);
        bad |= pbad[i];
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
        lo = __builtin_fmin(lo, __shfl_xor(lo, sh));
        hi = __builtin_fmax(hi, __shfl_xor(hi, sh));
        bad |= (uint32_t)__shfl_xor((int)bad, sh);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_lo[w] = lo; s_hi[w] = hi; s_bad[w] = bad; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < kF64Threads / 64; i++) {
        lo = __builtin_fmin(lo, s_lo[i]);
        hi = __builtin_fmax(hi, s_hi[i]);
        bad |= s_bad[i];
    }
    uint32_t status = 0;
    double e2 = 0.0, iv = 0.0;
    if (bad) {
        status = kErrNonfinite;
    } else {
        const double range = hi - lo;
        double eb_abs;
        if (range > 0.0) eb_abs = eb * range;
        else {
            const double a = __builtin_fabs(hi);
            eb_abs = eb * (a > 0.0 ? a : 1.0);
        }
        e2 = 2.0 * eb_abs;
        iv = 1.0 / e2;
        if (!(e2 >= 2.2250738585072014e-308) || !finite64(e2) || !finite64(iv) || !(iv > 0.0)) {
            status = kErrEbRange;
            e2 = 0.0;
            iv = 0.0;
        }
    }
    *reinterpret_cast<float*>(out + kOffEbx2) = (float)e2;
    *reinterpret_cast<float*>(out + kOffInv) = (float)iv;
    *reinterpret_cast<float*>(out + kOffVmin) = (float)lo;
    *reinterpret_cast<float*>(out + kOffVmax) = (float)hi;
    *reinterpret_cast<double*>(out + kOffEbx2F64) = e2;
    *reinterpret_cast<double*>(out + kOffInvF64) = iv;
    if (status) {
        *reinterpret_cast<uint32_t*>(out + kOffStatus) = status;
        *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off;
        reinterpret_cast<Scratch*>(out + g.scratch_off)->pre_status = status;
    }
}

// q = (int32) rint(x * inv) in double, round half to even, into the integer
// buffer; NaN/Inf and |x * inv| >= 2^31 set the status bits and end the
// pipeline (the compression kernel sees pre_status).
__global__ __launch_bounds__(kF64Threads) void k_prequant64(const double* __restrict__ x, int64_t n,
                                                           uint8_t* __restrict__ out, Geom g)
{
    __shared__ uint32_t s_err[kF64Threads / 64];
    Scratch* scr = reinterpret_cast<Scratch*>(out + g.scratch_off);
    if (scr->pre_status) return;  // set before this launch: uniform
    const double inv = *reinterpret_cast<const double*>(out + kOffInvF64);
    int32_t* q = reinterpret_cast<int32_t*>(out + g.q_off);
    uint32_t err = 0;
    auto quant = [&](double v) -> int32_t {
        if (!finite64(v)) { err |= kErrNonfinite; return 0; }
        const double p = v * inv;
        if (!(__builtin_fabs(p) < 2147483648.0)) { err |= kErrEbRange; return 0; }
        return (int32_t)__builtin_rint(p);
    };
    const int64_t stride = (int64_t)gridDim.x * kF64Threads;
    const int64_t tid = (int64_t)blockIdx.x * kF64Threads + threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;  // q's buffer is 256-aligned
    const int64_t n4 = vec ? n / 4 : 0;
    for (int64_t i = tid; i < n4; i += stride) {
        const fz_f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const fz_f64x2*>(x) + 2 * i);
        const fz_f64x2 b = __builtin_nontemporal_load(reinterpret_cast<const fz_f64x2*>(x) + 2 * i + 1);
        *reinterpret_cast<int4*>(q + 4 * i) = make_int4(quant(a.x), quant(a.y), quant(b.x), quant(b.y));
    }
    for (int64_t k = 4 * n4 + tid; k < n; k += stride) q[k] = quant(x[k]);
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) err |= (uint32_t)__shfl_xor((int)err, sh);
    if ((threadIdx.x & 63) == 0) s_err[threadIdx.x >> 6] = err;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kF64Threads / 64; i++) err |= s_err[i];
        if (err) {
            atomicOr(reinterpret_cast<uint32_t*>(out + kOffStatus), err);
            // every failing block writes the same size: the header alone
            *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off;
        }
    }
}

// The pre_status of k_compress must see the errors of a pass that wrote the
// integers (fp64 prequantization, the field-global faces): a second tiny
// kernel copies the header's status there (a failed block cannot know that
// the others finished).
__global__ void k_pre_status(uint8_t* __restrict__ out, Geom g)
{
    if (threadIdx.x == 0) {
        const uint32_t st = *reinterpret_cast<const uint32_t*>(out + kOffStatus);
        if (st) reinterpret_cast<Scratch*>(out + g.scratch_off)->pre_status = st;
    }
}

hipError_t launch_pre_status(uint8_t* out, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL(k_pre_status, dim3(1), dim3(64), 0, st, out, g);
    return hipGetLastError();
}

hipError_t launch_f64_front(const double* x, uint8_t* out, const Geom& g, int mode, double eb, hipStream_t st)
{
    const int64_t n = g.n[0] * g.n[1] * g.n[2];
    hipError_t e;
    if (mode == FZ_EB_REL) {
        int64_t blocks = (n / 2 + kF64Threads - 1) / kF64Threads;
        blocks = blocks < 1 ? 1 : blocks > kMinmaxBlocks ? kMinmaxBlocks : blocks;
        hipLaunchKernelGGL(k_minmax64, dim3((unsigned)blocks), dim3(kF64Threads), 0, st, x, n, out, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_params64, dim3(1), dim3(kF64Threads), 0, st, out, g, eb, (int)blocks);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int64_t blocks = (n / 4 + kF64Threads - 1) / kF64Threads;
    blocks = blocks < 1 ? 1 : blocks > 4096 ? 4096 : blocks;
    hipLaunchKernelGGL(k_prequant64, dim3((unsigned)blocks), dim3(kF64Threads), 0, st, x, n, out, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_pre_status(out, g, st);
}

// ------------------------------------------------------------ decompression
template <int RANK, bool VEC4>
__global__ __launch_bounds__(64, 2) void k_decompress64(const uint8_t* __restrict__ s, uint64_t sb, double* __restrict__ y,
                                                     Geom g, uint32_t* d_err)
{
    __shared__ __attribute__((aligned(16))) float tile[kTileFloats64];
    decompress_chunk_any<RANK, VEC4>(s, sb, y, g, d_err, blockIdx.x, threadIdx.x, tile);
}

__global__ void k_clear_err(uint32_t* p)
{
    if (threadIdx.x == 0) *p = 0u;
}

template <int RANK, bool VEC4>
static hipError_t launch_rank64(const uint8_t* s, uint64_t sb, double* y, const Geom& g, uint32_t* d_err, hipStream_t st)
{
    hipLaunchKernelGGL((k_decompress64<RANK, VEC4>), dim3((unsigned)g.n_chunks), dim3(64), 0, st, s, sb, y, g, d_err);
    return hipGetLastError();
}

hipError_t launch_decompress_f64(const uint8_t* s, uint64_t sb, double* y, const Geom& g, uint32_t* d_err,
                                 hipStream_t st)
{
    if (d_err) {
        hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(64), 0, st, d_err);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const bool vec4 = (reinterpret_cast<uintptr_t>(y) & 15) == 0 && (g.rank == 1 || (g.n[g.rank - 1] & 3) == 0);
    switch (g.rank * 2 + (vec4 ? 1 : 0)) {
        case 7: return launch_rank64<3, true>(s, sb, y, g, d_err, st);
        case 6: return launch_rank64<3, false>(s, sb, y, g, d_err, st);
        case 5: return launch_rank64<2, true>(s, sb, y, g, d_err, st);
        case 4: return launch_rank64<2, false>(s, sb, y, g, d_err, st);
        case 3: return launch_rank64<1, true>(s, sb, y, g, d_err, st);
        default: return launch_rank64<1, false>(s, sb, y, g, d_err, st);
    }
}

}  // namespace fz
