// fz_decompress_dev.hpp -- device code of the decompressor, shared by the
// per-field kernel (fz_decompress.hip) and the batched one (fz_batch.hip).
//
// The inverse of the compression pass (Sec. 4.4 calls the two pipelines
// symmetric).  One wave per chunk sweeps its steps in order.  Per step each
// lane loads word t of its nonzero bricks (their positions follow from the bit
// flags by popcount and mbcnt, Sec. 3.4) two steps before it computes them;
// it undoes the bitshuffle with the same in-register transpose, decodes the
// sign-magnitude codes (Sec. 3.2), and inverts the Lorenzo predictor as
// inclusive prefix sums: along the patch in registers, across lanes for the
// carries, and along the sweep dimension with the previous step kept in
// registers.  Then it dequantizes (one fp32 multiply, Sec. 2.3) and stores.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fz_device.hpp"
#include "fz_format.hpp"

namespace fz {

// dtype: 0 for an fp32 output, 1 for fp64; predictor: the header byte 15
// the caller handles (0 chunk-local Lorenzo, 1 field-global); s_bytes: the
// bytes readable at s (at least the header, table and flags, checked on the
// host)
__device__ __forceinline__ uint32_t check_header(const uint8_t* __restrict__ s, const Geom& g, int rank, int dtype,
                                                 int predictor, uint64_t s_bytes)
{
    // the whole header at once, as 32-bit words, and every check on them
    // without an early exit: the loads are uniform and issued together (one
    // wait), where byte loads behind branches would each wait in turn
    const uint32_t* hw = reinterpret_cast<const uint32_t*>(s);
    uint32_t w[kHeaderBytes / 4];
#pragma unroll
    for (int i = 0; i < kHeaderBytes / 4; i++) w[i] = hw[i];
    auto byte_at = [&](int off) { return (w[off / 4] >> (8 * (off % 4))) & 0xFFu; };
    auto u64_at = [&](int off) { return (uint64_t)w[off / 4] | ((uint64_t)w[off / 4 + 1] << 32); };
    bool bad = byte_at(kOffDtype) != (uint32_t)dtype || byte_at(kOffRank) != (uint32_t)rank ||
               byte_at(kOffEbMode) > (dtype ? 1u : 2u) || byte_at(kOffPredictor) != (uint32_t)predictor;
    if (dtype) {  // 2 eb as a normal, finite double
        const double e2 = __longlong_as_double((long long)u64_at(kOffEbx2F64));
        bad |= !(e2 >= 2.2250738585072014e-308 && e2 <= 1.7976931348623157e308);
    }
    const float st = __uint_as_float(w[kOffEbx2 / 4]);  // the point-wise mode's step: an integer in [2, 2^24)
    bad |= byte_at(kOffEbMode) == 2 && (!(st >= 2.0f && st < 16777216.0f) || st != __builtin_floorf(st));
#pragma unroll
    for (int i = 0; i < 3; i++) bad |= u64_at(kOffDims + 8 * i) != (uint64_t)g.n[i];
    bad |= w[kOffNChunks / 4] != (uint32_t)g.n_chunks;
    const uint64_t total = u64_at(kOffTotal);
    bad |= total < (uint64_t)g.payload_off || ((total - g.payload_off) & 15) != 0 || total > s_bytes;
    // the codes in the order of their precedence
    return w[kOffMagic / 4] != kMagic ? 6u                                                          // FZ_ERR_STREAM
         : w[kOffVersion / 4] != ((uint32_t)kVersion | ((uint32_t)kHeaderBytes << 16)) ? 7u  // FZ_ERR_VERSION
         : w[kOffStatus / 4] != 0u ? 8u                                                      // FZ_ERR_STATUS
         : bad ? 6u : 0u;
}

// Sign-magnitude decode (Sec. 3.2).  The transpose ran with plane 15 (the
// signs) cleared, so P[i] holds the magnitudes of codes i and i+16; bit m of
// `sgn` is the sign of code m.  d = (m ^ s) - s with s = 0 or -1.
__device__ __forceinline__ void decode_codes(const uint32_t (&P)[16], uint32_t sgn, int (&d)[32])
{
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int slo = (int)(sgn << (31 - i)) >> 31, shi = (int)(sgn << (15 - i)) >> 31;
        const int mlo = (int)(P[i] & 0xFFFFu), mhi = (int)(P[i] >> 16);
        d[i] = (mlo ^ slo) - slo;
        d[i + 16] = (mhi ^ shi) - shi;
    }
}

// Replace escaped cells (code 0x8000) by their logged deltas.  Pairs are in
// code-index order: this step's pairs follow the `seen` earlier ones.
__device__ __forceinline__ uint32_t apply_escapes(const uint32_t (&P)[16], uint32_t sgn, int (&d)[32],
                                                  const uint32_t* __restrict__ pairs, uint32_t nout, uint32_t& seen,
                                                  uint32_t n0, int lane)
{
    uint32_t emask = 0;  // the escape code 0x8000: sign set, magnitude 0
#pragma unroll
    for (int i = 0; i < 16; i++) {
        emask |= ((P[i] & 0xFFFFu) == 0u ? 1u : 0u) << i;
        emask |= ((P[i] >> 16) == 0u ? 1u : 0u) << (i + 16);
    }
    emask &= sgn;
    const int cnt = __popc(emask);
    const int incl = wave_incl_scan(cnt, lane);
    const uint32_t total = (uint32_t)__shfl(incl, 63);
    uint32_t pos = seen + (uint32_t)(incl - cnt);
    uint32_t bad = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if ((emask >> i) & 1u) {
            if (pos < nout && pairs[2 * pos] == n0 + (uint32_t)lane * kPatchCodes + i) d[i] = (int)pairs[2 * pos + 1];
            else bad = 1;
            pos++;
        }
    }
    seen += total;
    return bad;
}

// Dequantization (Sec. 2.3): q * 2eb in the output's precision (one fp32 or
// one fp64 multiply), or in the point-wise relative mode (fp32 only) the
// inverse of the bit-pattern transform with the stream's step.
template <bool PW, typename T>
__device__ __forceinline__ T dequant(int q, T ebx2, uint32_t step)
{
    if constexpr (std::is_integral_v<T>) return q;  // the integers themselves (field-global predictor)
    else if constexpr (PW) return pw_dequant(q, step);
    else return (T)q * ebx2;
}

// the 32-bit pattern an fp32 or integer output value leaves in the LDS tile
template <bool PW, typename T>
__device__ __forceinline__ float tile_val(int q, T ebx2, uint32_t step)
{
    if constexpr (std::is_integral_v<T>) return __int_as_float(q);
    else return dequant<PW>(q, ebx2, step);
}

template <int CNT, bool VEC4, bool PW, typename T>
__device__ __forceinline__ void store_run(T* __restrict__ p, const int* q, T ebx2, uint32_t step)
{
    if constexpr (VEC4 && std::is_integral_v<T>) {
#pragma unroll
        for (int j = 0; j < CNT / 4; j++)
            *reinterpret_cast<int4*>(p + 4 * j) = make_int4(q[4 * j], q[4 * j + 1], q[4 * j + 2], q[4 * j + 3]);
    } else if constexpr (VEC4 && sizeof(T) == 4) {
#pragma unroll
        for (int j = 0; j < CNT / 4; j++)
            *reinterpret_cast<float4*>(p + 4 * j) =
                make_float4(dequant<PW>(q[4 * j], ebx2, step), dequant<PW>(q[4 * j + 1], ebx2, step),
                            dequant<PW>(q[4 * j + 2], ebx2, step), dequant<PW>(q[4 * j + 3], ebx2, step));
    } else if constexpr (VEC4) {
#pragma unroll
        for (int j = 0; j < CNT / 2; j++)
            *reinterpret_cast<double2*>(p + 2 * j) =
                make_double2(dequant<PW>(q[2 * j], ebx2, step), dequant<PW>(q[2 * j + 1], ebx2, step));
    } else {
#pragma unroll
        for (int j = 0; j < CNT; j++) p[j] = dequant<PW>(q[j], ebx2, step);
    }
}

template <int CNT, bool PW, typename T>
__device__ __forceinline__ void store_run_masked(T* __restrict__ p, const int* q, T ebx2, uint32_t step, int valid)
{
#pragma unroll
    for (int j = 0; j < CNT; j++)
        if (j < valid) p[j] = dequant<PW>(q[j], ebx2, step);
}

// Decompress chunk c of a field with one wave (lane = 0..63; the workgroup is
// that one wave).  `tile` is kTileFloats of LDS.  A stream that fails a check
// writes an fz_status code to *d_err (if given) and leaves the chunk's output
// untouched.  No byte at or past s + s_bytes is read: the header's total is
// checked against s_bytes, and every chunk's payload against the total.
// LDS tile of one step: 3-D, 32 rows of 64 values with a row pitch of 68;
// 2-D and 1-D, the step's 2048 values in order with 4 floats of padding after
// every 32 (both paddings spread a wave's 16-byte accesses over the banks)
constexpr int kTilePitch = 68;

// Orders one wave's LDS accesses to its own tile (writes before the reads of
// other lanes, reads before the next rewrite): the compiler may not move
// memory operations across it, and the wave waits for its LDS operations.
// A workgroup barrier is not needed (no other wave touches the tile) and not
// possible where the waves of a workgroup run different numbers of steps.
__device__ __forceinline__ void wave_lds_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}
constexpr int kTileFloats = 2048 + 4 * (2048 / 32);
static_assert(32 * kTilePitch <= kTileFloats, "the 3-D tile fits");
__device__ __forceinline__ int run_slot(int i) { return i + 4 * (i >> 5); }

// Store one 2-D or 1-D step from its LDS tile (filled by the caller):
// instruction i writes values 256 i .. 256 i + 255 of the step, a run of 1 KiB
// of whole lines, streamed out.  Values 1024 r .. 1024 r + 1023 start at byte
// r * row_bytes from `base`: the step's second row in 2-D, 4096 in 1-D (one
// contiguous run).
__device__ __forceinline__ void store_tile_runs(const float* tile, void* base, uint32_t row_bytes, int lane)
{
    wave_lds_sync();  // orders the tile's writes before its reads
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, -1, kBufferFlags);
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const float4 v = *reinterpret_cast<const float4*>(tile + run_slot(256 * i + 4 * lane));
        const fz_u32x4 w = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
        const uint32_t soff = (uint32_t)(i >> 2) * row_bytes + 1024u * (uint32_t)(i & 3);
        __builtin_amdgcn_raw_buffer_store_b128(w, rs, 16u * (uint32_t)lane, soff, kCacheStreamStore);
    }
    wave_lds_sync();  // the tile is rewritten by the next step
}

// The same for a 2-D step of a chunk cut by the field's edge: `rows` (1 or
// 2) rows of `cols` values (a multiple of 4) from `base`, row pitch `nx`
// values; pieces outside the field are dropped by the resource's range
// (offset past it), and the stores are plain, as the lines are partly written.
__device__ __forceinline__ void store_tile_runs_edge(const float* tile, void* base, uint32_t nx, uint32_t rows,
                                                     uint32_t cols, int lane)
{
    wave_lds_sync();  // orders the tile's writes before its reads
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)(4u * ((rows - 1) * nx + cols)), kBufferFlags);
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const float4 v = *reinterpret_cast<const float4*>(tile + run_slot(256 * i + 4 * lane));
        const fz_u32x4 w = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
        const uint32_t row = (uint32_t)(i >> 2), col = 256u * (uint32_t)(i & 3) + 4u * (uint32_t)lane;
        const uint32_t voff = row < rows && col < cols ? 4u * (row * nx + col) : 0x80000000u;
        __builtin_amdgcn_raw_buffer_store_b128(w, rs, voff, 0u, 0);
    }
    wave_lds_sync();  // the tile is rewritten by the next step
}

// The fp64 output's tiles (twice the words; the caller's LDS holds
// kTileFloats64 floats): 3-D rows of 64 doubles with a pitch of 68 doubles;
// 2-D and 1-D runs of the step's 2048 doubles with 2 doubles of padding after
// every 16.  Every store instruction writes whole 512-byte rows (3-D) or
// 1 KiB of one row (2-D, 1-D), streamed out.
constexpr int kTilePitch64 = 68;  // doubles
constexpr int kTileFloats64 = 2 * (2048 + 2 * (2048 / 16));
static_assert(2 * 32 * kTilePitch64 <= kTileFloats64, "the 3-D fp64 tile fits");
__device__ __forceinline__ int run_slot64(int i) { return i + 2 * (i >> 4); }

__device__ __forceinline__ void store_nt2(double* p, double a, double b)
{
    const fz_f64x2 v = {a, b};
    __builtin_nontemporal_store(v, reinterpret_cast<fz_f64x2*>(p));
}

// 2-D / 1-D: instruction i writes doubles 128 i .. 128 i + 127 of the step;
// doubles 1024 r .. start at element r * row_elems from `base`
__device__ __forceinline__ void store_tile_runs64(const double* tile, double* base, int64_t row_elems, int lane)
{
    wave_lds_sync();  // orders the tile's writes before its reads
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const double2 v = *reinterpret_cast<const double2*>(tile + run_slot64(128 * i + 2 * lane));
        store_nt2(base + (int64_t)(i >> 3) * row_elems + 128 * (i & 7) + 2 * lane, v.x, v.y);
    }
    wave_lds_sync();  // the tile is rewritten by the next step
}

// 3-D: inclusive prefix of one plane of deltas along x, then y (the lane's
// 4x8 patch at rows 4 py.., columns 8 px..): inside the patch, with the carry
// across the lanes 8 apart (DPP and lane swaps) along x and across lanes -1,
// -2, -4 (a shift inside the 16-lane row) along y.
__device__ __forceinline__ void plane_prefix3(int (&d)[32], int lane)
{
    const int py = lane & 7;
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
        for (int cc = 1; cc < 8; cc++) d[8 * r + cc] += d[8 * r + cc - 1];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int ex_ = excl_scan_stride8(d[8 * r + 7], lane);
#pragma unroll
        for (int cc = 0; cc < 8; cc++) d[8 * r + cc] += ex_;
    }
#pragma unroll
    for (int r = 1; r < 4; r++)
#pragma unroll
        for (int cc = 0; cc < 8; cc++) d[8 * r + cc] += d[8 * (r - 1) + cc];
#pragma unroll
    for (int cc = 0; cc < 8; cc++) {
        const int C = d[24 + cc];
        int inc = C;
        int tv = row_shr<1>(inc);
        inc += py >= 1 ? tv : 0;
        tv = row_shr<2>(inc);
        inc += py >= 2 ? tv : 0;
        tv = row_shr<4>(inc);
        inc += py >= 4 ? tv : 0;
        const int ex_ = inc - C;
#pragma unroll
        for (int r = 0; r < 4; r++) d[8 * r + cc] += ex_;
    }
}

// 2-D: inclusive prefix along x of one row held as 16 values per lane (lane
// l has columns 16 l .. 16 l + 15)
__device__ __forceinline__ void row_prefix2(int* d, int lane)
{
#pragma unroll
    for (int cc = 1; cc < 16; cc++) d[cc] += d[cc - 1];
    const int tot = d[15];
    const int ex_ = wave_incl_scan(tot, lane) - tot;
#pragma unroll
    for (int cc = 0; cc < 16; cc++) d[cc] += ex_;
}

// Decompress chunk c of a field.  NW = 1: one wave (the workgroup) runs
// every layer.  NW = 2 or 4: the chunk's workgroup has NW waves, and wave
// `wave` runs layers 4/NW * wave .. (a field with few chunks, whose
// latency is set by a chunk's serial steps).  The prefix sums along the step
// dimension need what the layers below contributed: each wave first decodes
// its layers once and sums their deltas over the steps; the in-plane prefix of
// that sum is its contribution to the carry (the prefix is linear), left in
// `xch` (LDS, NW x 2048 ints).  After a workgroup barrier, wave w adds those of
// waves 0 .. w-1 to get its starting carry, then runs its layers as the single
// wave would.
template <int RANK, bool VEC4, bool PW, typename T, int NW>
__device__ __forceinline__ void decompress_chunk(const uint8_t* __restrict__ s, uint64_t s_bytes, T* __restrict__ y,
                                                 const Geom& g, uint32_t* d_err, int64_t c, int lane, float* tile,
                                                 int wave, int* xch)
{
    constexpr bool SPLIT = NW > 1;
    constexpr bool F64 = sizeof(T) == 8;
    constexpr bool INT = std::is_integral_v<T>;
    const uint32_t hdr_err = check_header(s, g, RANK, F64 ? 1 : 0, INT ? 1 : 0, s_bytes);
    if (hdr_err) {
        if (c == 0 && lane == 0 && d_err) atomicCAS(d_err, 0u, hdr_err);
        return;
    }
    const T ebx2 = INT ? (T)1
                 : F64 ? (T)*reinterpret_cast<const double*>(s + kOffEbx2F64)
                       : (T)*reinterpret_cast<const float*>(s + kOffEbx2);
    const uint32_t step = PW ? (uint32_t)ebx2 : 0u;  // the point-wise mode's step (checked by check_header)
    const uint64_t total = *reinterpret_cast<const uint64_t*>(s + kOffTotal);
    const uint64_t payload_units = (total - g.payload_off) / 16;
    const uint32_t* tab = reinterpret_cast<const uint32_t*>(s + g.table_off + 8 * c);
    const uint32_t off = tab[0], nout = tab[1];
    const uint64_t* F = reinterpret_cast<const uint64_t*>(s + g.flags_off + (int64_t)kFlagBytesPerChunk * c);
    int64_t org[3], ext[3];
    chunk_box(g, c, org, ext);
    const int L = layers_of(RANK, ext[0]);
    uint32_t nnz = 0;
    for (int i = 0; i < kLayers * kPlanes; i++) nnz += __popcll(F[i]);
    // the table is the exclusive prefix sum of the chunks' units (Sec. 3.4):
    // this chunk's offset plus its units (from the flags' popcounts and its
    // escape count) is the next chunk's offset, or the payload's end; with
    // chunk 0 at offset 0, every chunk lies inside the payload
    const uint64_t next = c + 1 < g.n_chunks ? (uint64_t)tab[2] : payload_units;
    bool bad = nout > (uint32_t)kChunkOutlierCap || (uint64_t)off + nnz + (nout + 1) / 2 != next || (c == 0 && off != 0);
    for (int i = L * kPlanes; i < kLayers * kPlanes; i++) bad |= F[i] != 0;
    if (bad) {
        if (lane == 0 && d_err) atomicCAS(d_err, 0u, 6u);
        return;
    }
    bool edge = false;
#pragma unroll
    for (int i = 0; i < 3; i++) edge |= ext[i] < g.box[i];

    const uint4* pay = reinterpret_cast<const uint4*>(s + g.payload_off);
    const uint32_t* pairs = reinterpret_cast<const uint32_t*>(pay + off + nnz);
    uint32_t seen = 0, esc_bad = 0;
    // the chunk's bricks through a buffer resource based at its payload (reads
    // past its nonzero bricks return 0, never another chunk's bytes)
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint4*>(pay + off), (short)0, (int)(16u * nnz), kBufferFlags);
    {
        // The bricks are read a few words per step over the chunk's 16 steps:
        // touch all their lines now (64 lines per instruction), so that the
        // later steps' loads find them in the caches instead of HBM.  The
        // words land in 256 bytes of LDS that nothing reads: a load into LDS
        // holds no register and nothing waits for it (the first step's wait
        // for its own words, issued after these, covers them in order).
        __shared__ uint32_t touch_dump[64];
        for (uint32_t o = 8192u * (uint32_t)wave; o < 16u * nnz; o += (uint32_t)NW * 8192u)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)touch_dump, 4,
                                                     o + 128u * (uint32_t)lane, 0, 0, 0);
    }

    // per-step brick words: plane b of this lane's brick holds word t of
    // step 4k + t at byte voff[b] + 4t of the chunk's payload.  A zero brick
    // gets an offset beyond the resource's range, where the load returns 0
    // without touching memory: every load is issued unconditionally, so the
    // wait for one step's words never has to cover the next step's loads.
    constexpr uint32_t kZeroBrick = 0x80000000u;
    uint32_t voff[16];
    uint32_t cur = 0;
    int k0 = 0, k1 = L;  // the layers this wave runs
    auto layer_offsets = [&](int k) {  // past the wave's last layer: all bricks zero
#pragma unroll
        for (int b = 0; b < 16; b++) {
            const uint64_t f = k < k1 ? F[k * kPlanes + b] : 0ull;
            voff[b] = ((f >> lane) & 1ull) ? 16u * (cur + mbcnt(f)) : kZeroBrick;
            cur += (uint32_t)__popcll(f);
        }
    };
    auto load_words = [&](int t, uint32_t (&w)[16]) {
#pragma unroll
        for (int b = 0; b < 16; b++) w[b] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff[b] + 4u * t, 0u, 0);
    };

    // per-rank geometry of this lane's patch
    const int py = lane & 7, px = lane >> 3;
    int carry3[32];   // 3-D: previous plane's q of this patch
    int carry2[16];   // 2-D: previous row's q of this patch
    int carry1 = 0;   // 1-D: q just before the current step
#pragma unroll
    for (int i = 0; i < 32; i++) carry3[i] = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) carry2[i] = 0;

    if constexpr (SPLIT) {
        k0 = (kLayers / NW) * wave;
        k1 = k0 + kLayers / NW < L ? k0 + kLayers / NW : L;
        // bricks and escape pairs of the layers below this one (the pairs are
        // in code-index order: those with an index below the layer's first)
        for (int i = 0; i < (k0 < L ? k0 : L) * kPlanes; i++) cur += (uint32_t)__popcll(F[i]);
        if (nout && k0 > 0) {
            const uint32_t first = (uint32_t)(4 * k0) * kStepCodes;
            uint32_t n = 0;
            for (uint32_t j = (uint32_t)lane; j < nout; j += 64) n += pairs[2 * j] < first ? 1u : 0u;
#pragma unroll
            for (int sh = 32; sh > 0; sh >>= 1) n += (uint32_t)__shfl_xor((int)n, sh);
            seen = n;
        }
        if (k0 < L) {
            // pass 1: the deltas of the wave's layers summed over their steps,
            // then their in-plane prefix (3-D: 32 per lane; 2-D: 16 per lane,
            // both rows of each step; 1-D: the total)
            const uint32_t cur0 = cur;
            int acc[32];
#pragma unroll
            for (int i = 0; i < 32; i++) acc[i] = 0;
            uint32_t seen1 = seen;
#pragma unroll 1
            for (int k = k0; k < k1; k++) {
                layer_offsets(k);
                uint32_t Wp[4][16];
#pragma unroll
                for (int t = 0; t < 4; t++) load_words(t, Wp[t]);
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    uint32_t P[16];
#pragma unroll
                    for (int b = 0; b < 15; b++) P[b] = Wp[t][b];
                    const uint32_t sgn = Wp[t][15];
                    P[15] = 0u;
                    transpose16(P);
                    int d[32];
                    decode_codes(P, sgn, d);
                    if (nout)
                        esc_bad |= apply_escapes(P, sgn, d, pairs, nout, seen1, (uint32_t)(4 * k + t) * kStepCodes, lane);
#pragma unroll
                    for (int i = 0; i < 32; i++) acc[i] += d[i];
                }
            }
            cur = cur0;
            int* xw = xch + 2048 * wave;
            if (RANK == 3) {
                plane_prefix3(acc, lane);
#pragma unroll
                for (int i = 0; i < 32; i++) xw[64 * i + lane] = acc[i];
            } else if (RANK == 2) {
#pragma unroll
                for (int cc = 0; cc < 16; cc++) acc[cc] += acc[16 + cc];
                row_prefix2(acc, lane);
#pragma unroll
                for (int cc = 0; cc < 16; cc++) xw[64 * cc + lane] = acc[cc];
            } else {
                int tot = 0;
#pragma unroll
                for (int i = 0; i < 32; i++) tot += acc[i];
#pragma unroll
                for (int sh = 32; sh > 0; sh >>= 1) tot += __shfl_xor(tot, sh);
                if (lane == 0) xw[0] = tot;
            }
        }
        __syncthreads();  // every wave reaches it: the checks above are the same for the whole chunk
        if (k0 >= L) return;
        for (int j = 0; j < wave; j++) {
            const int* xj = xch + 2048 * j;
            if (RANK == 3) {
#pragma unroll
                for (int i = 0; i < 32; i++) carry3[i] += xj[64 * i + lane];
            } else if (RANK == 2) {
#pragma unroll
                for (int cc = 0; cc < 16; cc++) carry2[cc] += xj[64 * cc + lane];
            } else {
                carry1 += xj[0];
            }
        }
    }

    // The words of a step are loaded two steps ahead: the wait for them then
    // leaves the previous step's stores outstanding (the counter of
    // outstanding vector memory operations covers stores too, in issue order).
    // W[t] holds the words of step t of a layer.  Every load is issued
    // unconditionally, so no register that a load is still filling is ever
    // copied at a join: iteration k = -1 loads zero bricks at t = 0, 1 and
    // layer 0's first words at t = 2, 3; the last layer loads the zero
    // bricks of the layer after it.
    uint32_t W[4][16];
#pragma unroll
    for (int b = 0; b < 16; b++) voff[b] = kZeroBrick;
    for (int k = k0 - 1; k < k1; k++) {
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (t == 2) layer_offsets(k + 1);  // the last load of layer k was issued at t = 1
            load_words(t < 2 ? t + 2 : t - 2, W[(t + 2) & 3]);
            __builtin_amdgcn_sched_barrier(0);
            const int st = 4 * k + t;
            const int64_t step_lo = RANK == 3 ? st : RANK == 2 ? 2 * st : (int64_t)kStepCodes * st;
            if (k < k0 || step_lo >= ext[0]) continue;
            uint32_t P[16];
#pragma unroll
            for (int b = 0; b < 15; b++) P[b] = W[t][b];
            const uint32_t sgn = W[t][15];  // plane 15: the signs
            P[15] = 0u;
            transpose16(P);
            int d[32];
            decode_codes(P, sgn, d);
            if (nout) esc_bad |= apply_escapes(P, sgn, d, pairs, nout, seen, (uint32_t)st * kStepCodes, lane);

            if (RANK == 3) {
                plane_prefix3(d, lane);
                // prefix along z: previous plane of the same patch
#pragma unroll
                for (int i = 0; i < 32; i++) {
                    d[i] += carry3[i];
                    carry3[i] = d[i];
                }
                const int64_t z = org[0] + st, y0 = org[1] + 4 * py, x0 = org[2] + 8 * px;
                if (edge && !(VEC4 && !F64 && 32 * 4 * g.n[2] < 0x80000000ll)) {
                    const int ey = clampi(ext[1] - 4 * py, 0, 4), ex = clampi(ext[2] - 8 * px, 0, 8);
#pragma unroll
                    for (int r = 0; r < 4; r++)
                        if (r < ey) store_run_masked<8, PW>(y + ((z * g.n[1] + y0 + r) * g.n[2] + x0), d + 8 * r, ebx2, step, ex);
                } else if constexpr (VEC4 && !F64) {
                    // the plane goes through LDS so that every store instruction
                    // writes 4 whole rows of 64 values (a lane's own 4x8 patch
                    // would give each instruction half-filled 32-byte pieces)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        float* t = tile + (4 * py + r) * kTilePitch + 8 * px;
                        *reinterpret_cast<float4*>(t) =
                            make_float4(tile_val<PW, T>(d[8 * r], ebx2, step), tile_val<PW, T>(d[8 * r + 1], ebx2, step),
                                        tile_val<PW, T>(d[8 * r + 2], ebx2, step), tile_val<PW, T>(d[8 * r + 3], ebx2, step));
                        *reinterpret_cast<float4*>(t + 4) =
                            make_float4(tile_val<PW, T>(d[8 * r + 4], ebx2, step), tile_val<PW, T>(d[8 * r + 5], ebx2, step),
                                        tile_val<PW, T>(d[8 * r + 6], ebx2, step), tile_val<PW, T>(d[8 * r + 7], ebx2, step));
                    }
                    wave_lds_sync();  // orders the tile's writes before its reads
                    T* plane = y + (z * g.n[1] + org[1]) * g.n[2] + org[2];
                    if (!edge) {
                        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(plane, (short)0, -1, kBufferFlags);
                        // offsets stay below 2^32: 32 rows of a contiguous extent below 2^25
                        const uint32_t voff = 4u * ((uint32_t)(lane >> 4) * (uint32_t)g.n[2] + 4u * (lane & 15));
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            const float4 v = *reinterpret_cast<const float4*>(tile + (4 * i + (lane >> 4)) * kTilePitch +
                                                                              4 * (lane & 15));
                            const fz_u32x4 w = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                                                __float_as_uint(v.w)};
                            __builtin_amdgcn_raw_buffer_store_b128(w, rs, voff, 16u * (uint32_t)i * (uint32_t)g.n[2],
                                                                   kCacheStreamStore);
                        }
                    } else {
                        // a chunk cut by the field's edge (its rows hold whole 16-byte pieces): the
                        // pieces outside the field get an offset past the resource's range, where
                        // the store is dropped; plain stores, as the rows' lines are partly written
                        const uint32_t rows = (uint32_t)ext[1], cols = (uint32_t)ext[2], nx = (uint32_t)g.n[2];
                        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                            plane, (short)0, (int)(4u * ((rows - 1) * nx + cols)), kBufferFlags);
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            const float4 v = *reinterpret_cast<const float4*>(tile + (4 * i + (lane >> 4)) * kTilePitch +
                                                                              4 * (lane & 15));
                            const fz_u32x4 w = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                                                __float_as_uint(v.w)};
                            const uint32_t row = 4u * i + (lane >> 4), col = 4u * (lane & 15);
                            const uint32_t voff = row < rows && col < cols ? 4u * (row * nx + col) : 0x80000000u;
                            __builtin_amdgcn_raw_buffer_store_b128(w, rs, voff, 0u, 0);
                        }
                    }
                    wave_lds_sync();  // the tile is rewritten by the next step
                } else if constexpr (VEC4 && F64) {
                    // through LDS as above: every store writes 2 whole rows of 64 doubles
                    double* t64 = reinterpret_cast<double*>(tile);
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        double* t = t64 + (4 * py + r) * kTilePitch64 + 8 * px;
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            *reinterpret_cast<double2*>(t + 2 * j) =
                                make_double2(dequant<PW>(d[8 * r + 2 * j], ebx2, step),
                                             dequant<PW>(d[8 * r + 2 * j + 1], ebx2, step));
                    }
                    wave_lds_sync();  // orders the tile's writes before its reads
                    T* base = y + (z * g.n[1] + org[1]) * g.n[2] + org[2];
#pragma unroll
                    for (int i = 0; i < 16; i++) {
                        const int row = 2 * i + (lane >> 5), col = 2 * (lane & 31);
                        const double2 v = *reinterpret_cast<const double2*>(t64 + row * kTilePitch64 + col);
                        store_nt2(base + (int64_t)row * g.n[2] + col, v.x, v.y);
                    }
                    wave_lds_sync();  // the tile is rewritten by the next step
                } else {
#pragma unroll
                    for (int r = 0; r < 4; r++) store_run<8, VEC4, PW>(y + ((z * g.n[1] + y0 + r) * g.n[2] + x0), d + 8 * r, ebx2, step);
                }
            } else if (RANK == 2) {
                row_prefix2(d, lane);
                row_prefix2(d + 16, lane);
#pragma unroll
                for (int cc = 0; cc < 16; cc++) {
                    d[cc] += carry2[cc];
                    d[16 + cc] += d[cc];
                    carry2[cc] = d[16 + cc];
                }
                const int64_t yy = org[0] + 2 * st, x0 = org[1] + 16 * lane;
                if (edge && !(VEC4 && !F64 && 2 * 4 * g.n[1] < 0x80000000ll)) {
                    const int ex = clampi(ext[1] - 16 * lane, 0, 16);
                    store_run_masked<16, PW>(y + (yy * g.n[1] + x0), d, ebx2, step, ex);
                    if (2 * st + 1 < ext[0]) store_run_masked<16, PW>(y + ((yy + 1) * g.n[1] + x0), d + 16, ebx2, step, ex);
                } else if constexpr (VEC4 && !F64) {
                    // through LDS, so that every store writes 1 KiB of one row
#pragma unroll
                    for (int r = 0; r < 2; r++)
#pragma unroll
                        for (int j = 0; j < 4; j++) {
                            const int* q = d + 16 * r + 4 * j;
                            *reinterpret_cast<float4*>(tile + run_slot(1024 * r + 16 * lane + 4 * j)) =
                                make_float4(tile_val<PW, T>(q[0], ebx2, step), tile_val<PW, T>(q[1], ebx2, step),
                                            tile_val<PW, T>(q[2], ebx2, step), tile_val<PW, T>(q[3], ebx2, step));
                        }
                    // row offsets stay below 2^32: the contiguous extent is below 2^25
                    if (!edge) store_tile_runs(tile, y + (yy * g.n[1] + org[1]), 4u * (uint32_t)g.n[1], lane);
                    else store_tile_runs_edge(tile, y + (yy * g.n[1] + org[1]), (uint32_t)g.n[1],
                                              (uint32_t)min((int64_t)2, ext[0] - 2 * st), (uint32_t)ext[1], lane);
                } else if constexpr (VEC4 && F64) {
                    double* t64 = reinterpret_cast<double*>(tile);
#pragma unroll
                    for (int r = 0; r < 2; r++)
#pragma unroll
                        for (int j = 0; j < 8; j++) {
                            const int* q = d + 16 * r + 2 * j;
                            *reinterpret_cast<double2*>(t64 + run_slot64(1024 * r + 16 * lane + 2 * j)) =
                                make_double2(dequant<PW>(q[0], ebx2, step), dequant<PW>(q[1], ebx2, step));
                        }
                    store_tile_runs64(t64, y + (yy * g.n[1] + org[1]), g.n[1], lane);
                } else {
                    store_run<16, VEC4, PW>(y + (yy * g.n[1] + x0), d, ebx2, step);
                    store_run<16, VEC4, PW>(y + ((yy + 1) * g.n[1] + x0), d + 16, ebx2, step);
                }
            } else {
#pragma unroll
                for (int m = 1; m < 32; m++) d[m] += d[m - 1];
                const int tot = d[31];
                const int ex_ = wave_incl_scan(tot, lane) - tot + carry1;
#pragma unroll
                for (int m = 0; m < 32; m++) d[m] += ex_;
                carry1 = __builtin_amdgcn_readlane(d[31], 63);
                const int64_t x0 = org[0] + (int64_t)kStepCodes * st + kPatchCodes * lane;
                if (edge) {
                    const int valid = clampi(ext[0] - ((int64_t)kStepCodes * st + kPatchCodes * lane), 0, 32);
                    store_run_masked<32, PW>(y + x0, d, ebx2, step, valid);
                } else if constexpr (VEC4 && !F64) {
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        const int* q = d + 4 * j;
                        *reinterpret_cast<float4*>(tile + run_slot(32 * lane + 4 * j)) =
                            make_float4(tile_val<PW, T>(q[0], ebx2, step), tile_val<PW, T>(q[1], ebx2, step),
                                        tile_val<PW, T>(q[2], ebx2, step), tile_val<PW, T>(q[3], ebx2, step));
                    }
                    store_tile_runs(tile, y + (org[0] + (int64_t)kStepCodes * st), 4096u, lane);
                } else if constexpr (VEC4 && F64) {
                    double* t64 = reinterpret_cast<double*>(tile);
#pragma unroll
                    for (int j = 0; j < 16; j++) {
                        const int* q = d + 2 * j;
                        *reinterpret_cast<double2*>(t64 + run_slot64(32 * lane + 2 * j)) =
                            make_double2(dequant<PW>(q[0], ebx2, step), dequant<PW>(q[1], ebx2, step));
                    }
                    store_tile_runs64(t64, y + (org[0] + (int64_t)kStepCodes * st), 1024, lane);
                } else {
                    store_run<32, VEC4, PW>(y + x0, d, ebx2, step);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // every escape code had its pair, and (the wave that ran the last layer)
    // no pair is left over
    if (nout && (esc_bad || (k1 == L && seen != nout))) {
        if (lane == 0 && d_err) atomicCAS(d_err, 0u, 6u);
    }
}

// Decompress chunk c with the stream's quantizer (the mode byte is uniform:
// one of the two bodies runs).  NW > 1: the form with NW waves per chunk
// (fp32 output only), `tile` this wave's own tile and `xch` the workgroup's
// carry exchange.
template <int RANK, bool VEC4, int NW = 1, typename T>
__device__ __forceinline__ void decompress_chunk_any(const uint8_t* __restrict__ s, uint64_t s_bytes,
                                                     T* __restrict__ y, const Geom& g, uint32_t* d_err, int64_t c,
                                                     int lane, float* tile, int wave = 0, int* xch = nullptr)
{
    static_assert(NW == 1 || std::is_same_v<T, float>, "the split forms write fp32 through fp32 tiles");
    static_assert(NW == 1 || NW == 2 || NW == 4, "a chunk's 4 layers are shared evenly");
    if constexpr (sizeof(T) == 8 || std::is_integral_v<T>) {
        // fp64 (grid modes only), or the integers of a field-global stream
        // (dequantized after the carries, in any mode)
        decompress_chunk<RANK, VEC4, false, T, 1>(s, s_bytes, y, g, d_err, c, lane, tile, 0, nullptr);
    } else {
        // the mode byte from its (uniform, scalar-loaded) header word
        const uint32_t mode = (reinterpret_cast<const uint32_t*>(s)[kOffEbMode / 4] >> (8 * (kOffEbMode % 4))) & 0xFFu;
        if (mode == 2) decompress_chunk<RANK, VEC4, true, T, NW>(s, s_bytes, y, g, d_err, c, lane, tile, wave, xch);
        else decompress_chunk<RANK, VEC4, false, T, NW>(s, s_bytes, y, g, d_err, c, lane, tile, wave, xch);
    }
}

}  // namespace fz
