// fz_device.hpp -- device helpers shared by the compression and
// decompression kernels of libfzmi (wave64 cross-lane moves, the in-register
// 16x16 bit transpose used for the bitshuffle, loaders).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fz_format.hpp"

namespace fz {

// raw buffer resources: dword 3 of the descriptor (gfx9 data format 32); a
// load at an offset of num_records bytes or more returns 0
constexpr int kBufferFlags = 0x00020000;
typedef uint32_t fz_u32x4 __attribute__((ext_vector_type(4)));
typedef float fz_f32x4 __attribute__((ext_vector_type(4)));
typedef double fz_f64x2 __attribute__((ext_vector_type(2)));

// cache policy of a buffer access: nontemporal (the nt bit).  Used where a
// kernel streams data it never touches again -- the reconstructed field,
// the range pass over the input -- so that the lines do not displace what
// the next kernel reads (measured: the 512^3 decompression 137 -> 116 us,
// the range pass about 9 us faster).  Only for stores that fill whole
// 128-byte lines per instruction: partial-line nontemporal stores lose the
// merging in L2 (measured 3-6x slower).
constexpr int kCacheStream = 2;
// the same for whole-line stores of data no kernel of the pipeline reads back
// soon (the reconstructed field): nt with system scope (sc1), which measured
// 116 -> 112 us against nt alone for back-to-back 512^3 decompressions (after
// a compression the two are within noise)
constexpr int kCacheStreamStore = 2 | 16;

// lane l receives lane l-1's value (DPP wave_shr:1).  Lane 0 receives an
// unspecified value: the compiler may leave the DPP destination of a lane
// without a source uninitialized, so callers mask it.
__device__ __forceinline__ int shift_up1_raw(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int shift_up1(int v, int lane)
{
    const int r = shift_up1_raw(v);
    return lane == 0 ? 0 : r;
}

// value of `v` held by lane - SH within the same row of 16 lanes (0 for the
// first SH lanes of a row)
template <int SH>
__device__ __forceinline__ int row_shr(int v)
{
    static_assert(SH >= 1 && SH <= 15, "row shift");
    return __builtin_amdgcn_update_dpp(0, v, 0x110 + SH, 0xf, 0xf, true);
}

// value of `v` held by lane (i + 8) mod 16 of the same 16-lane row
__device__ __forceinline__ int row_ror8(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false);
}

// Exclusive prefix sum of `v` over the 8 lanes with the same lane & 7, in
// the order of lane >> 3 (lanes 8 apart).  Within a 16-lane row the two
// halves are paired by DPP; the rows' totals are combined with the lane
// swaps (with both operands x, permlane16_swap gives the rows (x0, x0, x2,
// x2) and (x1, x1, x3, x3), permlane32_swap gives (x0, x1, x0, x1)).
__device__ __forceinline__ int excl_scan_stride8(int v, int lane)
{
    const int s1 = v + row_shr<8>(v);                   // upper half: its pair's inclusive sum
    const int r8 = row_ror8(s1);                         // on every lane: a lane shift under a branch
    const int u = (lane & 8) ? s1 : r8;                  // would read inactive lanes; the row's total
    const auto p = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
    const int a = (int)p[0];                             // rows: R0, R0, R2, R2
    const int c = a + (int)p[1];                         // rows: R0+R1, R0+R1, R2+R3, R2+R3
    const auto q = __builtin_amdgcn_permlane32_swap((uint32_t)c, (uint32_t)c, false, false);
    const int row = lane >> 4;
    int o = (row & 1) ? a : 0;                           // rows 1, 3: R0, R2
    o += (row & 2) ? (int)q[0] : 0;                      // rows 2, 3: + R0+R1
    return o + s1 - v;
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

__device__ __forceinline__ uint32_t absu(int d) { return d < 0 ? 0u - (uint32_t)d : (uint32_t)d; }

// how k_compress turns its input words into the integers q: fp32 values on
// the grid 2eb (Sec. 2.3), fp32 values through the point-wise relative
// transform, or words that already hold q (fp64 input, prequantized by a
// pass of its own)
constexpr int kQuantGrid = 0, kQuantPw = 1, kQuantInt = 2;

// The quantizer a stream records.  step == 0: the 2eb grid of the ABS and REL
// modes, q = rint(x * inv).  step > 0: the point-wise relative mode, where
// the data's logarithmic transform is the float's bit pattern b (exponent and
// mantissa, a piecewise-linear log2 exact in integers) and q = sign(x) *
// floor((b + floor(step / 2)) / step).  inv is 0 in that mode, so x * inv
// flags exactly the non-finite inputs.
struct Quant {
    float inv;
    uint32_t step;
    uint32_t magic;  // floor(2^32 / step): the division by step as a multiply-high
};

__device__ __forceinline__ Quant quant_of(const uint8_t* hdr)
{
    Quant z;
    z.inv = *reinterpret_cast<const float*>(hdr + kOffInv);
    const bool pw = hdr[kOffEbMode] == 2;
    z.step = pw ? (uint32_t)*reinterpret_cast<const float*>(hdr + kOffEbx2) : 0u;
    z.magic = pw ? (uint32_t)(0x100000000ull / (uint64_t)z.step) : 0u;
    return z;
}

// q of the point-wise relative mode.  n < 2^32, so the multiply-high estimate
// is floor(n / step) or one less, and one compare corrects it (Granlund and
// Montgomery's division by an invariant integer).
__device__ __forceinline__ int pw_quant(float x, const Quant& z)
{
    const uint32_t bits = __float_as_uint(x);
    const uint32_t n = (bits & 0x7FFFFFFFu) + (z.step >> 1);
    uint32_t a = __umulhi(n, z.magic);
    a += (n - a * z.step >= z.step) ? 1u : 0u;
    return (bits >> 31) ? -(int)a : (int)a;
}

// its inverse: the float with the sign of q and the bits min(|q| * step, the
// largest finite float)
__device__ __forceinline__ float pw_dequant(int q, uint32_t step)
{
    const uint64_t m = (uint64_t)absu(q) * step;
    const uint32_t b = m > 0x7F7FFFFFull ? 0x7F7FFFFFu : (uint32_t)m;
    return __uint_as_float(b | (q < 0 ? 0x80000000u : 0u));
}

// one value through the stream's quantizer; acc flags NaN/Inf (and in the
// grid modes |x * inv| >= 2^31)
__device__ __forceinline__ int prequant(float v, const Quant& z, uint32_t& acc)
{
    const int q = prequant(v, z.inv, acc);
    return z.step ? pw_quant(v, z) : q;
}

typedef short fz_short2 __attribute__((ext_vector_type(2)));

// Sign-magnitude 16-bit codes of d[i] and d[i+16] packed into one word
// (Sec. 3.2: sign in the MSB, magnitude below), computed on the packed low
// halves with 16-bit lane arithmetic.  `dmin` / `dmax` collect the range of
// the deltas (one v_min3 / v_max3 per pair) so that one compare per step
// finds deltas outside [-32767, 32767], whose codes the escape path then
// replaces.
__device__ __forceinline__ void pack_codes(const int (&d)[32], uint32_t (&P)[16], int& dmin, int& dmax)
{
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const uint32_t x = __builtin_amdgcn_perm((uint32_t)d[i + 16], (uint32_t)d[i], 0x05040100u);
        const fz_short2 xs = __builtin_bit_cast(fz_short2, x);
        const fz_short2 mag = __builtin_elementwise_max(xs, (fz_short2)0 - xs);
        P[i] = __builtin_bit_cast(uint32_t, mag) | (x & 0x80008000u);
        dmax = max(dmax, max(d[i], d[i + 16]));
        dmin = min(dmin, min(d[i], d[i + 16]));
    }
}
constexpr uint32_t kEscapeLimit = 65534u;  // d + 32767 above this (as unsigned): an escape
constexpr int kMaxCodeDelta = 32767;

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

// the byte stage of the transpose: two byte permutes per pair of words
__device__ __forceinline__ void tswap8(uint32_t& a, uint32_t& b)
{
    const uint32_t na = __builtin_amdgcn_perm(b, a, 0x06020400u);  // a0 b0 a2 b2
    const uint32_t nb = __builtin_amdgcn_perm(b, a, 0x07030501u);  // a1 b1 a3 b3
    a = na;
    b = nb;
}

__device__ __forceinline__ void transpose16(uint32_t (&P)[16])
{
#pragma unroll
    for (int i = 0; i < 8; i++) tswap8(P[i], P[i + 8]);
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

// a value that is the same on every lane, in scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void chunk_box(const Geom& g, int64_t c, int64_t org[3], int64_t ext[3])
{
    // chunk counts stay below 2^31, so 32-bit division suffices
    const uint32_t cc = (uint32_t)c, g2 = (uint32_t)g.grid[2], g1 = (uint32_t)g.grid[1];
    const uint32_t q2 = cc / g2;
    int64_t ci[3];
    ci[2] = cc - q2 * g2;
    ci[1] = q2 % g1;
    ci[0] = q2 / g1;
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
