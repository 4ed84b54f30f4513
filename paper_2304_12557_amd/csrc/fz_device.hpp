// fz_device.hpp -- device helpers shared by the compression and
// decompression kernels of libfzmi (wave64 cross-lane moves, the in-register
// 16x16 bit transpose used for the bitshuffle, loaders).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fz_format.hpp"

namespace fz {

// lane l receives lane l-1's value, lane 0 receives 0 (DPP wave_shr:1).
// Lane 0 is zeroed explicitly: the compiler may leave the DPP destination of
// a lane without a source uninitialized.
__device__ __forceinline__ int shift_up1(int v, int lane)
{
    const int r = __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
    return lane == 0 ? 0 : r;
}

// value of `v` held by lane `src` (any lane; indices wrap modulo 64)
__device__ __forceinline__ int lane_value(int v, int src)
{
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
        int t = lane_value(v, lane - sh);
        v += lane >= sh ? t : 0;
    }
    return v;
}

// Prequantization (Sec. 2.3): q = rint(x * inv), fp32 multiply then round
// half to even.  `acc` collects max(|p|) as shifted bits so that one compare
// per step detects NaN/Inf or |p| >= 2^31.
__device__ __forceinline__ int prequant(float v, float inv, uint32_t& acc)
{
    float p = v * inv;
    acc = max(acc, __float_as_uint(p) << 1);
    return (int)__builtin_rintf(p);
}
constexpr uint32_t kPrequantLimit = 0x4F000000u << 1;  // bits(2^31) << 1

__device__ __forceinline__ uint32_t absu(int d) { return d < 0 ? 0u - (uint32_t)d : (uint32_t)d; }

// Sign-magnitude 16-bit codes of d[i] and d[i+16] packed into one word
// (Sec. 3.2: sign in the MSB, magnitude below).  `macc` collects the largest
// magnitude so that one compare per step detects codes that need an escape.
__device__ __forceinline__ void pack_codes(const int (&d)[32], uint32_t (&P)[16], uint32_t& macc)
{
#pragma unroll
    for (int i = 0; i < 16; i++) {
        uint32_t m0 = absu(d[i]), m1 = absu(d[i + 16]);
        macc = max(macc, max(m0, m1));
        P[i] = (m0 & 0xFFFFu) | (m1 << 16) | (((uint32_t)d[i] >> 16) & 0x8000u) | ((uint32_t)d[i + 16] & 0x80000000u);
    }
}

// In-register bit transpose: on entry P[i] holds code i (low half) and code
// i+16 (high half); on exit P[b] bit m = bit b of code m (Sec. 3.3's
// bitshuffle of 32 codes).  The transform is its own inverse.
template <int S, uint32_t M>
__device__ __forceinline__ void tswap(uint32_t& a, uint32_t& b)
{
    uint32_t na = (a & M) | ((b << S) & ~M);
    uint32_t nb = ((a >> S) & M) | (b & ~M);
    a = na;
    b = nb;
}

__device__ __forceinline__ void transpose16(uint32_t (&P)[16])
{
#pragma unroll
    for (int i = 0; i < 8; i++) tswap<8, 0x00FF00FFu>(P[i], P[i + 8]);
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int i = (j & 3) | ((j & 4) << 1);
        tswap<4, 0x0F0F0F0Fu>(P[i], P[i + 4]);
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int i = (j & 1) | ((j & 6) << 1);
        tswap<2, 0x33333333u>(P[i], P[i + 2]);
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int i = 2 * j;
        tswap<1, 0x55555555u>(P[i], P[i + 1]);
    }
}

// order-preserving unsigned key of a float (-0 counts as +0)
__device__ __forceinline__ uint32_t float_key(float v)
{
    uint32_t b = __float_as_uint(v == 0.0f ? 0.0f : v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ void chunk_box(const Geom& g, int64_t c, int64_t org[3], int64_t ext[3])
{
    int64_t ci[3];
    ci[2] = c % g.grid[2];
    ci[1] = (c / g.grid[2]) % g.grid[1];
    ci[0] = c / (g.grid[2] * g.grid[1]);
#pragma unroll
    for (int i = 0; i < 3; i++) {
        org[i] = ci[i] * g.box[i];
        int64_t e = g.n[i] - org[i];
        ext[i] = e < g.box[i] ? e : g.box[i];
    }
}

// stored layers of a chunk whose extent along the step dimension is e
__device__ __forceinline__ int layers_of(int rank, int64_t e)
{
    const int64_t per = rank == 3 ? 4 : rank == 2 ? 8 : 8192;
    return (int)((e + per - 1) / per);
}

__device__ __forceinline__ int clampi(int64_t v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : (int)v);
}

}  // namespace fz
