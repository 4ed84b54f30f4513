// fz_ablation.hip -- the paper's per-kernel ablation pipeline (Sec. 4.5),
// rebuilt on MI355X to measure the same relative effects.
//
// The product compresses in one fused kernel.  The ablation instead runs the
// kernel split that the paper compares, on 3-D fields whose extents are
// multiples of the 16x32x64 chunk box, in the product's code geometry: a step
// is one z-plane (32 x 64) of a chunk, cut into 64 patches of 4 rows x 8
// columns.
//   pred-quant v1 : the original dual-quantization (Sec. 2.3): q = rint(x * inv)
//                   with inv = fp32(1 / (2 eb)) (one fp32 multiply, as the
//                   product's prequantization), chunk-local Lorenzo delta d; a code q' = d + r for -r < d < r,
//                   else code 0 and d written to a dense outlier array of one
//                   int32 per value (r = 512).
//   pred-quant v2 : the optimized one (Sec. 3.2): no shift, no outlier
//                   handling, a 16-bit sign-magnitude code (|d| > 32767 gives
//                   the escape code 0x8000, whose value this pipeline drops).
//   bitshuffle-mark v1 : two kernels: the bitshuffle writes each step's tile
//                   to HBM, the mark kernel reads it back for the flags.
//   bitshuffle-mark v2 : one kernel writes the tile and the flags.
//   prefix-sum-encode  : a scan of the per-step block counts, then the
//                   compaction of the nonzero blocks (Sec. 3.4), run on the
//                   tiles of either code version.
// Tile of a step (4 KB): word T[b*64 + p] holds bit b of the 32 codes of patch
// p (bit m = cell m; cell m is row m/8, column m%8 of the patch; patch p covers
// rows 4*(p%8).., columns 8*(p/8)..).  Block beta (16 B) = T[4*beta .. 4*beta+3]:
// plane beta/16 of 128 consecutive codes (Sec. 3.4).  Flags: 4 u64 per step,
// bit beta%64 of word beta/64.  The steps are numbered chunk-major, each chunk
// in z order.
#include <hip/hip_runtime.h>

#include "fz.h"
#include "fz_device.hpp"
#include "fz_format.hpp"

namespace fz {
namespace {

constexpr int kAblRadius = 512;
constexpr int kAblRows = 32, kAblCols = 64;  // one step of a 3-D chunk

struct AblGeom {
    int64_t n[3];   // field extents, slowest first
    int64_t gc[3];  // chunks per dimension
    int64_t steps;  // 16 per chunk
};

bool abl_geom(const fz_dims* d, AblGeom* g)
{
    if (!d || d->rank != 3) return false;
    const int64_t box[3] = {16, kAblRows, kAblCols};
    int64_t total = 1;
    for (int i = 0; i < 3; i++) {
        if (d->n[i] == 0 || d->n[i] % box[i] != 0 || d->n[i] > (1ull << 24)) return false;
        g->n[i] = (int64_t)d->n[i];
        g->gc[i] = g->n[i] / box[i];
        total *= g->n[i];
    }
    if (total >= (1ll << 36)) return false;
    g->steps = g->gc[0] * g->gc[1] * g->gc[2] * 16;
    return true;
}

// first element of step s (chunk-major, z order inside the chunk)
__device__ __forceinline__ int64_t step_origin(const AblGeom& g, int64_t s, int* zin)
{
    const int64_t c = s >> 4;
    *zin = (int)(s & 15);
    const int64_t cx = c % g.gc[2], cy = (c / g.gc[2]) % g.gc[1], cz = c / (g.gc[2] * g.gc[1]);
    return ((cz * 16 + *zin) * g.n[1] + cy * kAblRows) * g.n[2] + cx * kAblCols;
}

// One workgroup of 256 threads per chunk sweeps its 16 planes in z order:
// each plane is read once and prequantized into LDS, where it stays as the
// plane below the next one; each thread codes 8 cells of a plane, row-major.
template <int V>
__global__ __launch_bounds__(256) void k_abl_pq(const float* __restrict__ x, AblGeom g, float inv,
                                                uint16_t* __restrict__ codes, int32_t* __restrict__ outl)
{
    __shared__ int32_t qs[2][kAblRows][kAblCols];
    uint32_t acc = 0;
    for (int e = threadIdx.x; e < kAblRows * kAblCols; e += 256) qs[1][e / kAblCols][e % kAblCols] = 0;
    for (int zin = 0; zin < 16; zin++) {
        int z0;
        const int64_t base = step_origin(g, (int64_t)blockIdx.x * 16 + zin, &z0);
        int32_t (&qc)[kAblRows][kAblCols] = qs[zin & 1];
        const int32_t (&qp)[kAblRows][kAblCols] = qs[(zin & 1) ^ 1];
        for (int e = threadIdx.x; e < kAblRows * kAblCols; e += 256) {
            const int r = e / kAblCols, c = e % kAblCols;
            qc[r][c] = prequant(x[base + (int64_t)r * g.n[2] + c], inv, acc);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kAblRows * kAblCols; e += 256) {
            const int r = e / kAblCols, c = e % kAblCols;
            auto at = [&](const int32_t (&q)[kAblRows][kAblCols], int rr, int cc) -> uint32_t {
                return (rr >= 0 && cc >= 0) ? (uint32_t)q[rr][cc] : 0u;
            };
            // the 3-D Lorenzo difference in wrapping 32-bit arithmetic (the
            // plane below the chunk's first is zero)
            const uint32_t dz0 = at(qc, r, c) - at(qc, r, c - 1) - at(qc, r - 1, c) + at(qc, r - 1, c - 1);
            const uint32_t dz1 = at(qp, r, c) - at(qp, r, c - 1) - at(qp, r - 1, c) + at(qp, r - 1, c - 1);
            const int d = (int)(dz0 - dz1);
            const int64_t i = base + (int64_t)r * g.n[2] + c;
            if (V == 1) {
                if (d > -kAblRadius && d < kAblRadius) {  // the original kernel's branch
                    codes[i] = (uint16_t)(d + kAblRadius);
                    outl[i] = 0;
                } else {
                    codes[i] = 0;
                    outl[i] = d;
                }
            } else {
                const uint32_t m = absu(d);
                codes[i] = m <= 32767u ? (uint16_t)((d < 0 ? 0x8000u : 0u) | m) : (uint16_t)kEscape;
            }
        }
        __syncthreads();  // the next plane is written over the one below this one
    }
}

// this lane's patch of step s as 16 plane words (P[b] bit m = bit b of cell m)
__device__ __forceinline__ void load_patch_words(const uint16_t* __restrict__ codes, const AblGeom& g, int64_t s,
                                                 int lane, uint32_t (&P)[16])
{
    int zin;
    const int64_t base = step_origin(g, s, &zin);
    const int py = lane & 7, px = lane >> 3;
    uint16_t v[32];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint4 t = *reinterpret_cast<const uint4*>(codes + base + (int64_t)(4 * py + r) * g.n[2] + 8 * px);
        const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            v[8 * r + 2 * k] = (uint16_t)(w[k] & 0xFFFFu);
            v[8 * r + 2 * k + 1] = (uint16_t)(w[k] >> 16);
        }
    }
#pragma unroll
    for (int i = 0; i < 16; i++) P[i] = (uint32_t)v[i] | ((uint32_t)v[i + 16] << 16);
    transpose16(P);
}

// bitshuffle v1: one wave per step; the tile goes to HBM
__global__ __launch_bounds__(64) void k_abl_shuffle(const uint16_t* __restrict__ codes, AblGeom g,
                                                    uint32_t* __restrict__ tiles)
{
    const int lane = threadIdx.x;
    uint32_t P[16];
    load_patch_words(codes, g, blockIdx.x, lane, P);
    uint32_t* t = tiles + (int64_t)blockIdx.x * 1024;
#pragma unroll
    for (int b = 0; b < 16; b++) t[b * 64 + lane] = P[b];
}

// mark v1: one wave per step reads the tile back; lane l owns blocks l, l+64,
// l+128, l+192
__global__ __launch_bounds__(64) void k_abl_mark(const uint32_t* __restrict__ tiles, AblGeom g,
                                                 uint64_t* __restrict__ flags)
{
    const int lane = threadIdx.x;
    const uint4* t = reinterpret_cast<const uint4*>(tiles + (int64_t)blockIdx.x * 1024);
    uint64_t mine = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint4 blk = t[64 * j + lane];
        const uint64_t f = __ballot((blk.x | blk.y | blk.z | blk.w) != 0u);
        mine = lane == j ? f : mine;
    }
    if (lane < 4) flags[(int64_t)blockIdx.x * 4 + lane] = mine;
}

// ------------------------------------------------ ballot bitshuffle (Sec. 3.3)
// The paper's transpose: the codes of a tile sit in shared memory two to a
// 32-bit word, and a warp vote per bit gathers that bit of every thread's
// word into one word.  On wave64 one vote covers 64 lanes, so the step's codes
// are arranged for it: lane l takes cell l % 32 of patch 2k + l / 32 for the
// patch pairs k = 0..31, two pairs per word (pair 2w in the low half of word
// w, pair 2w + 1 in the high half).  The vote on bit i of word w then holds
// plane i % 16 of the pair 2w + i / 16: its low 32 bits are the plane word of
// the pair's first patch, its high 32 bits that of the second.  512 votes per
// step; each result is written into the lane that owns the patch.
constexpr int kAblRowWords = kAblCols / 2 + 1;  // 32 words of two codes per row, plus one of padding

// this lane's patch of step s as 16 plane words, by votes (the tile's codes
// pass through `buf`, this wave's 32 x 33 words of LDS)
__device__ __forceinline__ void ballot_patch_words(const uint16_t* __restrict__ codes, const AblGeom& g, int64_t s,
                                                   int lane, uint32_t* buf, uint32_t (&P)[16])
{
    int zin;
    const int64_t base = step_origin(g, s, &zin);
    // the step's 32 x 64 codes into LDS, row r in words r * 33 .. r * 33 + 31
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int e = 64 * j + lane, r = e >> 3, c8 = (e & 7) * 8;  // 8 codes per lane and load
        const uint4 t = *reinterpret_cast<const uint4*>(codes + base + (int64_t)r * g.n[2] + c8);
        uint32_t* d = buf + r * kAblRowWords + c8 / 2;
        d[0] = t.x; d[1] = t.y; d[2] = t.z; d[3] = t.w;
    }
    __syncthreads();
    const uint16_t* b16 = reinterpret_cast<const uint16_t*>(buf);
    const int m = lane & 31, half = lane >> 5;
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int pp = 2 * k + half;  // patch of this lane in pair k
        const int row = 4 * (pp & 7) + (m >> 3), col = 8 * (pp >> 3) + (m & 7);
        const uint32_t c = b16[2 * row * kAblRowWords + col];
        if (k & 1) w[k >> 1] |= c << 16;
        else w[k >> 1] = c;
    }
#pragma unroll
    for (int b = 0; b < 16; b++) P[b] = 0u;
#pragma unroll
    for (int ww = 0; ww < 16; ww++) {
#pragma unroll
        for (int i = 0; i < 32; i++) {
            const uint64_t v = __ballot((w[ww] >> i) & 1u);
            const int pair = 2 * ww + (i >> 4), b = i & 15;
            // the vote's halves go to lanes 2 pair and 2 pair + 1
            const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
            P[b] = lane == 2 * pair ? lo : lane == 2 * pair + 1 ? hi : P[b];
        }
    }
}

// bitshuffle v1 with votes: one wave per step; the tile goes to HBM
__global__ __launch_bounds__(64) void k_abl_shuffle_ballot(const uint16_t* __restrict__ codes, AblGeom g,
                                                           uint32_t* __restrict__ tiles)
{
    __shared__ uint32_t buf[kAblRows * kAblRowWords];
    const int lane = threadIdx.x;
    uint32_t P[16];
    ballot_patch_words(codes, g, blockIdx.x, lane, buf, P);
    uint32_t* t = tiles + (int64_t)blockIdx.x * 1024;
#pragma unroll
    for (int b = 0; b < 16; b++) t[b * 64 + lane] = P[b];
}

// flag words of a step from its 16 plane words in registers (block 16b + q
// covers the patches, i.e. lanes, 4q .. 4q + 3); lane j < 4 gets word j
__device__ __forceinline__ uint64_t step_flags(const uint32_t (&P)[16], int lane)
{
    uint64_t F[4] = {0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 16; b++) {
        uint64_t m = __ballot(P[b] != 0u);
        m |= m >> 1;
        m |= m >> 2;
        uint32_t f = 0;
#pragma unroll
        for (int q = 0; q < 16; q++) f |= (uint32_t)((m >> (4 * q)) & 1u) << q;
        F[b >> 2] |= (uint64_t)f << (16 * (b & 3));
    }
    return lane == 0 ? F[0] : lane == 1 ? F[1] : lane == 2 ? F[2] : F[3];
}

// bitshuffle-mark v2 with votes
__global__ __launch_bounds__(64) void k_abl_shuffle_mark_ballot(const uint16_t* __restrict__ codes, AblGeom g,
                                                                uint32_t* __restrict__ tiles,
                                                                uint64_t* __restrict__ flags)
{
    __shared__ uint32_t buf[kAblRows * kAblRowWords];
    const int lane = threadIdx.x;
    uint32_t P[16];
    ballot_patch_words(codes, g, blockIdx.x, lane, buf, P);
    uint32_t* t = tiles + (int64_t)blockIdx.x * 1024;
#pragma unroll
    for (int b = 0; b < 16; b++) t[b * 64 + lane] = P[b];
    const uint64_t f = step_flags(P, lane);
    if (lane < 4) flags[(int64_t)blockIdx.x * 4 + lane] = f;
}

// bitshuffle-mark v2: the flags come from the words in registers
__global__ __launch_bounds__(64) void k_abl_shuffle_mark(const uint16_t* __restrict__ codes, AblGeom g,
                                                         uint32_t* __restrict__ tiles, uint64_t* __restrict__ flags)
{
    const int lane = threadIdx.x;
    uint32_t P[16];
    load_patch_words(codes, g, blockIdx.x, lane, P);
    uint32_t* t = tiles + (int64_t)blockIdx.x * 1024;
#pragma unroll
    for (int b = 0; b < 16; b++) t[b * 64 + lane] = P[b];
    const uint64_t f = step_flags(P, lane);
    if (lane < 4) flags[(int64_t)blockIdx.x * 4 + lane] = f;
}

// prefix sum: block counts per step -> exclusive offsets, in tiles of 8192
// steps, one workgroup each.  Pass 1: thread t counts the 8 consecutive steps
// 8t .. 8t+7 of its tile (16 loads in flight), the workgroup scans the 1024
// sums and writes the tile-local offsets and the tile total (to `tot`).
// Pass 2: each tile adds the totals of the tiles before it.
constexpr int kAblScanThreads = 1024, kAblScanPer = 8;
constexpr int64_t kAblScanTile = (int64_t)kAblScanThreads * kAblScanPer;

__global__ __launch_bounds__(kAblScanThreads) void k_abl_scan_local(const uint64_t* __restrict__ flags, int64_t steps,
                                                                     uint64_t* __restrict__ offsets,
                                                                     uint64_t* __restrict__ tot)
{
    __shared__ uint64_t s_wave[kAblScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * kAblScanTile + (int64_t)threadIdx.x * kAblScanPer;
    const int64_t n = s0 < steps ? min((int64_t)kAblScanPer, steps - s0) : 0;
    uint32_t cnt[kAblScanPer];
    const uint4* f = reinterpret_cast<const uint4*>(flags + 4 * s0);
#pragma unroll
    for (int k = 0; k < kAblScanPer; k++) {
        const int kk = k < n ? k : 0;  // loads stay inside the flags; out-of-range steps count 0
        const uint4 a = n > 0 ? f[2 * kk] : make_uint4(0, 0, 0, 0);
        const uint4 b = n > 0 ? f[2 * kk + 1] : make_uint4(0, 0, 0, 0);
        const uint32_t c = __popc(a.x) + __popc(a.y) + __popc(a.z) + __popc(a.w) + __popc(b.x) + __popc(b.y) +
                           __popc(b.z) + __popc(b.w);
        cnt[k] = k < n ? c : 0u;
    }
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kAblScanPer; k++) sum += cnt[k];
    uint64_t inc = sum;
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
        const uint64_t v = __shfl_up(inc, sh);
        inc += lane >= sh ? v : 0;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint64_t pos = inc - sum;
    for (int k = 0; k < w; k++) pos += s_wave[k];
#pragma unroll
    for (int k = 0; k < kAblScanPer; k++) {
        if (k < n) offsets[s0 + k] = pos;
        pos += cnt[k];
    }
    if (threadIdx.x == kAblScanThreads - 1) tot[blockIdx.x] = pos;
}

__global__ __launch_bounds__(kAblScanThreads) void k_abl_scan_fix(int64_t steps, const uint64_t* __restrict__ tot,
                                                                   uint64_t* __restrict__ offsets)
{
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) {
        uint64_t c = 0;
        for (unsigned i = 0; i < blockIdx.x; i++) c += tot[i];
        s_carry = c;
        if (blockIdx.x == gridDim.x - 1) offsets[steps] = c + tot[blockIdx.x];
    }
    __syncthreads();
    const uint64_t carry = s_carry;
    const int64_t s0 = (int64_t)blockIdx.x * kAblScanTile;
    for (int64_t i = threadIdx.x; i < kAblScanTile && s0 + i < steps; i += kAblScanThreads) offsets[s0 + i] += carry;
}

// encode: one wave per step copies its nonzero blocks, in block order, to
// 16 * offsets[s] bytes into the payload
__global__ __launch_bounds__(64) void k_abl_encode(const uint32_t* __restrict__ tiles,
                                                   const uint64_t* __restrict__ flags,
                                                   const uint64_t* __restrict__ offsets, uint4* __restrict__ out)
{
    const int lane = threadIdx.x;
    const int64_t s = blockIdx.x;
    const uint4* t = reinterpret_cast<const uint4*>(tiles + s * 1024);
    uint64_t pos = offsets[s];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint64_t f = flags[4 * s + j];
        if ((f >> lane) & 1ull) out[pos + mbcnt(f)] = t[64 * j + lane];
        pos += (uint64_t)__popcll(f);
    }
}

hipError_t done() { return hipGetLastError(); }

}  // namespace
}  // namespace fz

using namespace fz;

extern "C" {

int fz_abl_pred_quant(int version, const float* d_x, const fz_dims* dims, float inv, uint16_t* d_codes,
                      int32_t* d_outliers, void* stream)
{
    AblGeom g;
    if (!d_x || !d_codes || !abl_geom(dims, &g) || !(inv > 0.0f) || !__builtin_isfinite(inv)) return FZ_ERR_ARG;
    if (version != 1 && version != 2) return FZ_ERR_ARG;
    if (version == 1 && !d_outliers) return FZ_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (version == 1)
        hipLaunchKernelGGL(k_abl_pq<1>, dim3((unsigned)(g.steps / 16)), dim3(256), 0, st, d_x, g, inv, d_codes,
                           d_outliers);
    else
        hipLaunchKernelGGL(k_abl_pq<2>, dim3((unsigned)(g.steps / 16)), dim3(256), 0, st, d_x, g, inv, d_codes,
                           d_outliers);
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_abl_bitshuffle(const uint16_t* d_codes, const fz_dims* dims, uint32_t* d_tiles, void* stream)
{
    AblGeom g;
    if (!d_codes || !d_tiles || !abl_geom(dims, &g)) return FZ_ERR_ARG;
    hipLaunchKernelGGL(k_abl_shuffle, dim3((unsigned)g.steps), dim3(64), 0, static_cast<hipStream_t>(stream), d_codes,
                       g, d_tiles);
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_abl_mark(const uint32_t* d_tiles, const fz_dims* dims, uint64_t* d_flags, void* stream)
{
    AblGeom g;
    if (!d_tiles || !d_flags || !abl_geom(dims, &g)) return FZ_ERR_ARG;
    hipLaunchKernelGGL(k_abl_mark, dim3((unsigned)g.steps), dim3(64), 0, static_cast<hipStream_t>(stream), d_tiles, g,
                       d_flags);
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_abl_bitshuffle_ballot(const uint16_t* d_codes, const fz_dims* dims, uint32_t* d_tiles, void* stream)
{
    AblGeom g;
    if (!d_codes || !d_tiles || !abl_geom(dims, &g)) return FZ_ERR_ARG;
    hipLaunchKernelGGL(k_abl_shuffle_ballot, dim3((unsigned)g.steps), dim3(64), 0, static_cast<hipStream_t>(stream),
                       d_codes, g, d_tiles);
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_abl_bitshuffle_mark_ballot(const uint16_t* d_codes, const fz_dims* dims, uint32_t* d_tiles, uint64_t* d_flags,
                                  void* stream)
{
    AblGeom g;
    if (!d_codes || !d_tiles || !d_flags || !abl_geom(dims, &g)) return FZ_ERR_ARG;
    hipLaunchKernelGGL(k_abl_shuffle_mark_ballot, dim3((unsigned)g.steps), dim3(64), 0,
                       static_cast<hipStream_t>(stream), d_codes, g, d_tiles, d_flags);
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_abl_bitshuffle_mark(const uint16_t* d_codes, const fz_dims* dims, uint32_t* d_tiles, uint64_t* d_flags,
                           void* stream)
{
    AblGeom g;
    if (!d_codes || !d_tiles || !d_flags || !abl_geom(dims, &g)) return FZ_ERR_ARG;
    hipLaunchKernelGGL(k_abl_shuffle_mark, dim3((unsigned)g.steps), dim3(64), 0, static_cast<hipStream_t>(stream),
                       d_codes, g, d_tiles, d_flags);
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_abl_encode(const uint32_t* d_tiles, const uint64_t* d_flags, const fz_dims* dims, uint64_t* d_offsets,
                  void* d_out, void* stream)
{
    AblGeom g;
    if (!d_tiles || !d_flags || !d_offsets || !d_out || !abl_geom(dims, &g)) return FZ_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the tile totals wait at the start of d_out, which the compaction only
    // writes after both scan passes
    const int64_t tiles = (g.steps + kAblScanTile - 1) / kAblScanTile;
    uint64_t* tot = static_cast<uint64_t*>(d_out);
    hipLaunchKernelGGL(k_abl_scan_local, dim3((unsigned)tiles), dim3(kAblScanThreads), 0, st, d_flags, g.steps,
                       d_offsets, tot);
    if (done() != hipSuccess) return FZ_ERR_HIP;
    hipLaunchKernelGGL(k_abl_scan_fix, dim3((unsigned)tiles), dim3(kAblScanThreads), 0, st, g.steps, tot, d_offsets);
    if (done() != hipSuccess) return FZ_ERR_HIP;
    hipLaunchKernelGGL(k_abl_encode, dim3((unsigned)g.steps), dim3(64), 0, st, d_tiles, d_flags, d_offsets,
                       static_cast<uint4*>(d_out));
    return done() == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

}  // extern "C"
