// fz_compress_dev.hpp -- device code of the compression pipeline, shared by
// the per-field kernels (fz_compress.hip) and the batched ones (fz_batch.hip).
//
// The path of one chunk: a workgroup of 4 waves, wave k on layer k (4 steps),
// one lane per 32-code patch.  Per step a lane prequantizes its 32 fp32 values
// (Sec. 2.3), applies the Lorenzo difference on the integers (Sec. 2.3 / 3.2;
// the previous step sits in the same lane's registers, the other neighbours
// come from adjacent lanes), maps the deltas to sign-magnitude 16-bit codes
// (Sec. 3.2) with packed 16-bit arithmetic, and bit-transposes the 32 codes in
// registers (the bitshuffle of Sec. 3.3).  After its 4 steps a lane holds 16
// bricks (one per bit plane); a ballot per plane gives the bit flags of the
// zero-block encoder (Sec. 3.4), and the nonzero bricks are compacted into
// the workgroup's staging slot with coalesced 16-byte writes.  A layer whose
// deltas need escapes is computed again out of line; its (index, delta) pairs
// are written after the workgroup barrier, once every layer's count is known,
// straight to their place behind the chunk's bricks.  A chunk cut by the
// field's edge runs the same code; the codes of its cells outside the field
// are cleared afterwards.  One chunk later, when
// a look-back over the published chunk sizes (the device-wide prefix sum of
// Sec. 3.4) has given the chunk its offset, the slot is copied there.
#pragma once
#include <hip/hip_runtime.h>

#include "fz_device.hpp"
#include "fz_format.hpp"
#include "fz_kernels.hpp"

namespace fz {

struct EscapeLog {
    uint32_t* pairs;  // null: count only; else the layer's (index, delta) pairs in the payload
    int count;        // escapes seen so far in this layer
    int room;         // pairs that may be written (what the chunk's allowance leaves the layer)
};

// Slow path of a step with at least one escape: codes whose delta does not
// fit in 15 bits become 0x8000 and their (code index, delta) pair is logged
// in code-index order (lane-major, then cell).
__device__ __forceinline__ void log_escapes(const int (&d)[32], uint32_t (&P)[16], EscapeLog& log, uint32_t n0, int lane)
{
    uint32_t emask = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) emask |= ((uint32_t)d[i] + 32767u > kEscapeLimit ? 1u : 0u) << i;
    const int cnt = __popc(emask);
    const int incl = wave_incl_scan(cnt, lane);
    const int total = __shfl(incl, 63);
    int pos = log.count + incl - cnt;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if ((emask >> i) & 1u) {
            if (log.pairs && pos < log.room)
                *reinterpret_cast<uint2*>(log.pairs + 2 * pos) = make_uint2(n0 + (uint32_t)lane * kPatchCodes + i, (uint32_t)d[i]);
            pos++;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
        if ((emask >> i) & 1u) P[i] = (P[i] & 0xFFFF0000u) | kEscape;
        if ((emask >> (i + 16)) & 1u) P[i] = (P[i] & 0x0000FFFFu) | (kEscape << 16);
    }
    log.count += total;
}

// codes -> escapes -> bit planes, shared tail of every rank's step.  The fast
// pass (ESC = false) only reports that a step needs escapes; the layer is then
// redone by the logging pass (ESC = true), which rewrites those codes.
template <bool ESC>
__device__ __forceinline__ bool finish_step(const int (&d)[32], uint32_t (&P)[16], EscapeLog& log, uint32_t n0, int lane)
{
    int dmin = 0, dmax = 0;
    pack_codes(d, P, dmin, dmax);
    const bool esc = __ballot(dmax > kMaxCodeDelta || dmin < -kMaxCodeDelta) != 0;
    if (ESC && esc) log_escapes(d, P, log, n0, lane);
    transpose16(P);
    return esc;
}

// prequantize 32 values; `facc` tracks max |p| with NaN propagating
// (v_maximum3_f32), so one compare per step (!(facc < 2^31)) finds NaN, Inf
// or an overflowing product
template <int QM>
__device__ __forceinline__ void prequant32(const float (&v)[32], const Quant& z, float& facc, int (&q)[32])
{
    if constexpr (QM == kQuantInt) {  // the values are already the integers q (fp64 input)
#pragma unroll
        for (int i = 0; i < 32; i++) q[i] = __float_as_int(v[i]);
        return;
    }
    const float inv = z.inv;  // 0 in the point-wise mode: x * inv flags NaN/Inf there
#pragma unroll
    for (int i = 0; i < 32; i += 2) {
        const float p0 = v[i] * inv, p1 = v[i + 1] * inv;
        facc = __builtin_elementwise_maximum(facc, __builtin_elementwise_maximum(__builtin_fabsf(p0), __builtin_fabsf(p1)));
        if constexpr (QM == kQuantPw) {
            q[i] = pw_quant(v[i], z);
            q[i + 1] = pw_quant(v[i + 1], z);
        } else {
            q[i] = (int)__builtin_rintf(p0);
            q[i + 1] = (int)__builtin_rintf(p1);
        }
    }
}

// ------------------------------------------------------------------ loaders
// Loads go through a buffer resource whose base is the (uniform) first value
// of the step: a lane keeps one 32-bit byte offset for the whole chunk and
// the row offsets are uniform, so no 64-bit per-lane address is held in
// registers.  The resource's range ends at the field's last value, so a load
// past it returns 0 without touching memory.  A chunk cut by the field's edge
// is loaded exactly like an interior one: its cells outside the field read 0
// (past the end) or values of other chunks (the rest of a row, the next
// rows), and their deltas are set to 0 afterwards (mask_outside), while the
// delta of a cell inside the field only looks at cells inside it.
// (on = false: a range of 0, every load returns 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t step_rsrc(const float* __restrict__ x, const Geom& g,
                                                           const float* base, bool on = true)
{
    const int64_t left = 4 * (g.n[0] * g.n[1] * g.n[2] - (base - x));  // uniform
    const int range = !on || left <= 0 ? 0 : left >= 0xFFFFFFFFll ? -1 : (int)(uint32_t)left;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, range, kBufferFlags);
}

// CNT values from voff + soff; VEC4: in 16-byte loads, which need only 4-byte
// alignment and are range-checked per dword (the host's vec_loads); else one
// load per value.  NT: a nontemporal (streaming) load, for values this chunk
// reads only once.
template <int CNT, bool VEC4, bool NT = false>
__device__ __forceinline__ void load_run(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float* v)
{
    if (VEC4) {
#pragma unroll
        for (int j = 0; j < CNT / 4; j++) {
            const fz_u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16u * j, soff, NT ? kCacheStream : 0);
            v[4 * j] = __uint_as_float(t.x); v[4 * j + 1] = __uint_as_float(t.y);
            v[4 * j + 2] = __uint_as_float(t.z); v[4 * j + 3] = __uint_as_float(t.w);
        }
    } else {
#pragma unroll
        for (int j = 0; j < CNT; j++)
            v[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff + 4u * j, soff, NT ? kCacheStream : 0));
    }
}

// Per-chunk, per-lane geometry.  step_base() is uniform (scalar); lane
// offsets inside a step are 32-bit.
struct Lane {
    int64_t org[3], ext[3];
    int L;
    bool edge;
    uint32_t off;  // lane offset of its first value inside a step
};

template <int RANK>
__device__ __forceinline__ Lane lane_geo(const Geom& g, int64_t c, int lane)
{
    Lane l;
    chunk_box(g, c, l.org, l.ext);
    // the box is the same on every lane, but its divisions run on the vector
    // unit: copied to scalar registers, so that the loads' row offsets and
    // resources built from it stay scalar
#pragma unroll
    for (int i = 0; i < 3; i++) {
        l.org[i] = uniform64(l.org[i]);
        l.ext[i] = uniform64(l.ext[i]);
    }
    l.L = layers_of(RANK, l.ext[0]);
    l.edge = false;
#pragma unroll
    for (int i = 0; i < 3; i++) l.edge |= l.ext[i] < g.box[i];
    if (RANK == 3) {
        const int py = lane & 7, px = lane >> 3;
        l.off = (uint32_t)(4 * py * g.n[2] + 8 * px);
    } else if (RANK == 2) {
        l.off = (uint32_t)(16 * lane);
    } else {
        l.off = (uint32_t)(kPatchCodes * lane);
    }
    return l;
}

// first value of step s (3-D: plane s; 2-D: row 2s; 1-D: value 2048 s) of the chunk
template <int RANK>
__device__ __forceinline__ const float* step_base(const float* __restrict__ x, const Geom& g, const Lane& l, int64_t s)
{
    if (RANK == 3) return x + ((l.org[0] + s) * g.n[1] + l.org[1]) * g.n[2] + l.org[2];
    if (RANK == 2) return x + (l.org[0] + 2 * s) * g.n[1] + l.org[1];
    return x + l.org[0] + (int64_t)kStepCodes * s;
}

// load the lane's 32 values of step s (s = 4k-1 is the halo of layer k),
// through the step's ranged resource (step_rsrc; on = false: zeros).  NT: 3-D
// loads nontemporal (streaming).
template <int RANK, bool VEC4, bool NT>
__device__ __forceinline__ void load_step_as(const float* __restrict__ x, const Geom& g, const Lane& l, int64_t s,
                                             bool on, float (&v)[32])
{
    const float* b = step_base<RANK>(x, g, l, s);
    const __amdgpu_buffer_rsrc_t rs = step_rsrc(x, g, b, on);
    if (RANK == 3) {
        const int64_t nx = g.n[2];
#pragma unroll
        for (int r = 0; r < 4; r++) load_run<8, VEC4, NT>(rs, 4u * l.off, (uint32_t)(4 * r * nx), v + 8 * r);
    } else if (RANK == 2) {
        const int64_t nx = g.n[1];
#pragma unroll
        for (int r = 0; r < 2; r++) load_run<16, VEC4>(rs, 4u * l.off, (uint32_t)(4 * r * nx), v + 16 * r);
    } else {
        load_run<32, VEC4>(rs, 4u * l.off, 0u, v);
    }
}

// 3-D loads are nontemporal except for the top step of a layer (s mod 4 =
// 3), which the next layer's wave reads again as its halo in the same
// iteration and must find in the cache (measured: the 512^3 ABS compression
// 173 -> 166 us).  After unrolling, s mod 4 is a constant.  In 2-D and 1-D a
// lane's run spans 4 or 8 load instructions per line, and nontemporal loads
// there measured 6 % and 40 % slower: lines left before the rest of their run
// was read.
template <int RANK, bool VEC4>
__device__ __forceinline__ void load_step(const float* __restrict__ x, const Geom& g, const Lane& l, int64_t s,
                                          float (&v)[32])
{
    if ((s & 3) == 3) load_step_as<RANK, VEC4, false>(x, g, l, s, true, v);
    else load_step_as<RANK, VEC4, RANK == 3>(x, g, l, s, true, v);
}

// The lane's cells of step s inside the field, one bit per value of d (all
// set in a chunk not cut by the field's edge): 3-D, its rows r < ev and
// columns c < eh of a plane inside the field; 2-D, its columns c < eh of the
// step's rows inside the field; 1-D, its values inside the field.
template <int RANK>
__device__ __forceinline__ uint32_t keep_bits(const Lane& l, int64_t s, int lane)
{
    if (RANK == 3) {
        const int ev = clampi(l.ext[1] - 4 * (lane & 7), 0, 4), eh = clampi(l.ext[2] - 8 * (lane >> 3), 0, 8);
        const uint32_t cells = (uint32_t)((1ull << (8 * ev)) - 1ull) & (((1u << eh) - 1u) * 0x01010101u);
        return s < l.ext[0] ? cells : 0u;
    } else if (RANK == 2) {
        const uint32_t cols = (uint32_t)((1ull << clampi(l.ext[1] - 16 * lane, 0, 16)) - 1ull);
        return (2 * s < l.ext[0] ? cols : 0u) | (2 * s + 1 < l.ext[0] ? cols << 16 : 0u);
    } else {
        const int valid = clampi(l.ext[0] - ((int64_t)kStepCodes * s + l.off), 0, 32);
        return (uint32_t)((1ull << valid) - 1ull);
    }
}

// Deltas of the cells of step s outside the field set to 0 (the logging
// pass, which must not log an escape for such a cell).
template <int RANK>
__device__ __forceinline__ void mask_outside(int (&d)[32], const Lane& l, int64_t s, int lane)
{
    const uint32_t keep = keep_bits<RANK>(l, s, lane);
#pragma unroll
    for (int i = 0; i < 32; i++) d[i] &= __builtin_amdgcn_sbfe((int)keep, (uint32_t)i, 1u);
}

// ------------------------------------------------------------- one layer
// In-plane part of the Lorenzo difference, after the difference along the
// sweep dimension.  3-D: `a` is a plane difference; Dy then Dx give d.
__device__ __forceinline__ void inplane3(const int (&a)[32], int (&d)[32], int lane)
{
    const int py = lane & 7, px = lane >> 3;
    int b[32];
#pragma unroll
    for (int c = 0; c < 8; c++) {  // Dy; row 0 takes row 3 of lane-1 (0 for py == 0)
        const int up = shift_up1_raw(a[24 + c]);
        b[c] = a[c] - (py == 0 ? 0 : up);
    }
#pragma unroll
    for (int r = 1; r < 4; r++)
#pragma unroll
        for (int c = 0; c < 8; c++) b[8 * r + c] = a[8 * r + c] - a[8 * (r - 1) + c];
#pragma unroll
    for (int r = 0; r < 4; r++) {  // Dx; column 0 takes column 7 of lane-8 (0 for px == 0)
        const int left = lane_value(b[8 * r + 7], lane - 8);
        d[8 * r] = b[8 * r] - (px == 0 ? 0 : left);
#pragma unroll
        for (int c = 1; c < 8; c++) d[8 * r + c] = b[8 * r + c] - b[8 * r + c - 1];
    }
}

// 2-D: `b` holds the two row differences of the step (rows 2s, 2s+1); Dx
// gives d.
__device__ __forceinline__ void inplane2(const int (&b)[32], int (&d)[32], int lane)
{
#pragma unroll
    for (int r = 0; r < 2; r++) {  // Dx; column 0 takes column 15 of lane-1 (0 at lane 0)
        const int left = shift_up1_raw(b[16 * r + 15]);
        d[16 * r] = b[16 * r] - (lane == 0 ? 0 : left);
#pragma unroll
        for (int c = 1; c < 16; c++) d[16 * r + c] = b[16 * r + c] - b[16 * r + c - 1];
    }
}

// `h` holds the halo (3-D: the plane before the layer; 2-D: the two rows
// before it, of which the second is used; 1-D: unused) and `v` the first
// step, both loaded ahead of time.  The plane-b word of step t goes to
// Wl[(b * 4 + t) * 64 + lane] in LDS (brick (k, b, lane) = its 4 words) and
// nz[b] collects their OR for the flags.
// Returns whether some delta of the layer needs an escape (only the ESC pass
// logs them).
template <int RANK, bool VEC4, bool ESC, int QM = kQuantGrid>
__device__ __forceinline__ bool layer(const float* __restrict__ x, const Geom& g, const Lane& l, int k, Quant inv,
                                      int lane, float (&h)[32], float (&v)[32], uint32_t* Wl, uint32_t (&nz)[16],
                                      float& facc, EscapeLog& log)
{
    // the logging pass (ESC) keeps one copy of the step code: it runs rarely
    // and must not add to the register budget of the fast pass
    bool esc = false;
#pragma unroll
    for (int b = 0; b < 16; b++) nz[b] = 0u;
    // previous-step state: 3-D plane (32), 2-D row (16), 1-D last value (uniform)
    int qprev[32];
    int carry1 = 0;
    if (k == 0 || RANK == 1) {
#pragma unroll
        for (int i = 0; i < 32; i++) qprev[i] = 0;
        if (RANK == 1 && k > 0) {
            uint32_t dummy = 0;
            const float xh = x[l.org[0] + (int64_t)kStepCodes * 4 * k - 1];
            carry1 = QM == kQuantPw ? pw_quant(xh, inv) : QM == kQuantInt ? __float_as_int(xh) : prequant(xh, inv.inv, dummy);
        }
    } else if (RANK == 3) {
        prequant32<QM>(h, inv, facc, qprev);
    } else {
        int qh[32];
        prequant32<QM>(h, inv, facc, qh);
#pragma unroll
        for (int c = 0; c < 16; c++) qprev[c] = qh[16 + c];
    }
#pragma unroll ESC ? 1 : 4
    for (int t = 0; t < 4; t++) {
        const int s = 4 * k + t;
        float vn[32];
        if (t < 3) load_step<RANK, VEC4>(x, g, l, s + 1, vn);
        // keep the steps apart: the scheduler must not pull the next step's
        // arithmetic up to its loads, which would wait on them right away
        __builtin_amdgcn_sched_barrier(0);
        int q[32];
        prequant32<QM>(v, inv, facc, q);
        int d[32];
        if (RANK == 3) {
            int a[32];
#pragma unroll
            for (int i = 0; i < 32; i++) {
                a[i] = q[i] - qprev[i];  // Dz
                qprev[i] = q[i];
            }
            inplane3(a, d, lane);
        } else if (RANK == 2) {
            int b[32];
#pragma unroll
            for (int c = 0; c < 16; c++) {  // Dy against the previous row of the same lane
                b[c] = q[c] - qprev[c];
                b[16 + c] = q[16 + c] - q[c];
                qprev[c] = q[16 + c];
            }
            inplane2(b, d, lane);
        } else {
            const int left = shift_up1_raw(q[31]);
            d[0] = q[0] - (lane == 0 ? carry1 : left);
#pragma unroll
            for (int m = 1; m < 32; m++) d[m] = q[m] - q[m - 1];
            carry1 = __builtin_amdgcn_readlane(q[31], 63);
        }
        if (ESC) mask_outside<RANK>(d, l, s, lane);
        uint32_t P[16];
        esc |= finish_step<ESC>(d, P, log, (uint32_t)s * kStepCodes, lane);
#pragma unroll
        for (int bb = 0; bb < 16; bb++) {
            Wl[(bb * 4 + t) * 64 + lane] = P[bb];
            nz[bb] |= P[bb];
        }
        if (t < 3) {
#pragma unroll
            for (int i = 0; i < 32; i++) v[i] = vn[i];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return esc;
}

// Layer k swept downwards (fast path of odd layers, 2-D and 3-D).  An odd layer's halo is the top plane of the
// layer below it, and an even layer's halo the top plane of an odd layer; in
// this order each halo plane is loaded in the same iteration as by the wave
// that owns it, so the second load is served by the cache.  `h` holds the top
// step of the layer and `v` the one below it.  The deltas and words are those
// of the forward sweep; escapes are only detected (the out-of-line pass logs
// them in code order).
template <int RANK, bool VEC4, int QM = kQuantGrid>
__device__ __forceinline__ bool layer_rev(const float* __restrict__ x, const Geom& g, const Lane& l, int k, Quant inv,
                                          int lane, float (&h)[32], float (&v)[32], uint32_t* Wl, uint32_t (&nz)[16],
                                          float& facc, EscapeLog& log)
{
    static_assert(RANK >= 2, "the 1-D halo is one value");
    bool esc = false;
#pragma unroll
    for (int b = 0; b < 16; b++) nz[b] = 0u;
    int cq[32];  // q of the step being coded (3-D: its plane; 2-D: its two rows)
    prequant32<QM>(h, inv, facc, cq);
#pragma unroll
    for (int it = 0; it < 4; it++) {
        const int t = 3 - it, s = 4 * k + t;
        float vn[32];
        if (it < 3) load_step<RANK, VEC4>(x, g, l, s - 2, vn);  // s - 2 = 4k - 1 at it = 2: the halo
        __builtin_amdgcn_sched_barrier(0);
        int ql[32];  // q of step s - 1
        prequant32<QM>(v, inv, facc, ql);
        int d[32];
        if (RANK == 3) {
            int a[32];
#pragma unroll
            for (int i = 0; i < 32; i++) {
                a[i] = cq[i] - ql[i];  // Dz
                cq[i] = ql[i];
            }
            inplane3(a, d, lane);
        } else {
            int b[32];
#pragma unroll
            for (int c = 0; c < 16; c++) {  // Dy: row 2s against row 2s-1, row 2s+1 against row 2s
                b[c] = cq[c] - ql[16 + c];
                b[16 + c] = cq[16 + c] - cq[c];
            }
#pragma unroll
            for (int i = 0; i < 32; i++) cq[i] = ql[i];
            inplane2(b, d, lane);
        }
        uint32_t P[16];
        esc |= finish_step<false>(d, P, log, (uint32_t)s * kStepCodes, lane);
#pragma unroll
        for (int bb = 0; bb < 16; bb++) {
            Wl[(bb * 4 + t) * 64 + lane] = P[bb];
            nz[bb] |= P[bb];
        }
        if (it < 3) {
#pragma unroll
            for (int i = 0; i < 32; i++) v[i] = vn[i];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return esc;
}

// Whether layer k of a chunk is swept downwards.
template <int RANK>
__device__ __forceinline__ bool swept_down(int k)
{
    return RANK >= 2 && (k & 1);
}

// Load the first two steps that layer k of a chunk uses ahead of time: the
// halo and the first step (upwards), or the top two steps (downwards).
// Branch-free: both loads are always issued, and one that has nothing to
// read (no layer k, the halo of layer 0 or of a 1-D layer) gets a range of 0
// and returns zeros.  A branch here would merge the loads' uniform row
// offsets at its join, where the compiler keeps them in vector registers and
// then has to build a loop around every later load that uses them.  The
// halo or top step is the one another wave reads again (cached), the other
// one is streamed.
template <int RANK, bool VEC4>
__device__ __forceinline__ void prefetch(const float* __restrict__ x, const Geom& g, const Lane& l, int k,
                                         float (&h)[32], float (&v)[32], bool down = false)
{
    const bool live = k < l.L, dn = down && live;
    if (RANK == 1) {  // no halo step (a 1-D layer's halo is one value)
#pragma unroll
        for (int i = 0; i < 32; i++) h[i] = 0.0f;
    } else {
        load_step_as<RANK, VEC4, false>(x, g, l, dn ? 4 * k + 3 : 4 * k - 1, live && (dn || k > 0), h);
    }
    load_step_as<RANK, VEC4, RANK == 3>(x, g, l, dn ? 4 * k + 2 : 4 * k, live, v);
}

// Out-of-line layer pass for the uncommon case of a layer whose deltas need
// escapes (computed again with the escape codes).  It loads its own inputs, writes the layer's bricks to Wl, logs the
// escape pairs to `pairs` (at most `room` of them; null: count only) and
// returns (escape count << 32) | max-|p| bits.  The geometry is read from the copy
// in the scratch so that nothing large crosses the call.  It stays a real
// call: inlined, its registers would push the fast path into spills, while
// as a call the register saves happen only on this path.
template <int RANK, bool VEC4, int QM = kQuantGrid>
__device__ __noinline__ uint64_t layer_slow(const float* __restrict__ x, const uint8_t* scr,
                                            int64_t c, int k, Quant inv, int lane, uint32_t* Wl, uint32_t* pairs,
                                            int room)
{
    const Geom g = *reinterpret_cast<const Geom*>(scr + kScratchGeomOff);
    const Lane l = lane_geo<RANK>(g, c, lane);
    float h[32], v[32];
    prefetch<RANK, VEC4>(x, g, l, k, h, v);
    uint32_t nz[16];
    float facc = 0.0f;
    EscapeLog log{pairs, 0, room};
    layer<RANK, VEC4, true, QM>(x, g, l, k, inv, lane, h, v, Wl, nz, facc, log);
    return ((uint64_t)(uint32_t)log.count << 32) | __float_as_uint(facc);
}

// Rare path: a step saw NaN/Inf or |x*inv| >= 2^31.  Re-read the layer's
// cells and classify them the way the format defines the status bits
// (halo values belong to the previous layer, which reports them).
__device__ __forceinline__ uint32_t classify_errors(const float* __restrict__ x, const uint8_t* scr,
                                                 int64_t c, int k, Quant inv, int lane)
{
    const Geom g = *reinterpret_cast<const Geom*>(scr + kScratchGeomOff);
    int64_t o[3], e[3];
    chunk_box(g, c, o, e);
    uint32_t err = 0;
    for (int t = 0; t < 4; t++) {
        const int s = 4 * k + t;
        for (int m = 0; m < 32; m++) {
            int64_t r0 = 0, r1 = 0, r2 = 0;
            if (g.rank == 3) { r0 = s; r1 = 4 * (lane % 8) + m / 8; r2 = 8 * (lane / 8) + m % 8; }
            else if (g.rank == 2) { r0 = 2 * s + m / 16; r1 = 16 * lane + m % 16; }
            else { r0 = (int64_t)kStepCodes * s + kPatchCodes * lane + m; }
            if (r0 >= e[0] || r1 >= e[1] || r2 >= e[2]) continue;
            const float v = x[((o[0] + r0) * g.n[1] + o[1] + r1) * g.n[2] + o[2] + r2];
            if (!__builtin_isfinite(v)) err |= kErrNonfinite;
            else if (!(__builtin_fabsf(v * inv.inv) < 2147483648.0f)) err |= kErrEbRange;
        }
    }
    return err;
}


// ------------------------------------------------------------ one chunk
// Workgroup-shared state of a compression workgroup (4 waves, one chunk).
struct CompressLds {
    uint32_t err;
    uint32_t nnz[kLayers], nout[kLayers];
    uint32_t arrived;  // waves whose layer of the current chunk is done
    uint64_t ticket;
    uint64_t excl;  // offset of the chunk being placed (16-B units), from the look-back
    // per wave: the bricks of its layer (as plane-step words)
    uint32_t w[kLayers][kPlanes * 4 * 64];
};

// Payload size of the chunk in S (16-B units): its nonzero bricks, then its
// escape pairs padded to 16 bytes (none when the chunk holds more than
// kChunkOutlierCap escapes: the stream then carries the OUTLIER_CAP status).
__device__ __forceinline__ uint32_t chunk_units(const CompressLds& S)
{
    const uint32_t tn = S.nnz[0] + S.nnz[1] + S.nnz[2] + S.nnz[3];
    const uint32_t to = S.nout[0] + S.nout[1] + S.nout[2] + S.nout[3];  // each at most 8192: no overflow
    const uint32_t kept = to > (uint32_t)kChunkOutlierCap ? 0u : to;
    return tn + (kept + 1) / 2;
}

// Chunk state words are read and written with agent-scope atomics: the
// workgroups that publish and read them run on different XCDs, whose L2
// caches are not coherent with one another.
__device__ __forceinline__ void publish_state(uint64_t* p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t peek_state(const uint64_t* p)
{
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Tail of a wave's layer: the data-dependent status bits (NaN/Inf or an
// overflowing product, seen in facc), the flags of the
// zero-block encoder (one ballot per bit plane, F; lane b < 16 gets F[b] in
// `myflag`, which stage_chunk stores), and the layer's counts in S.  Returns
// the layer's escape count.
__device__ __forceinline__ int layer_flags(const float* __restrict__ x, const uint8_t* __restrict__ scr, const Geom& g,
                                           int64_t c, int wave, int lane, Quant inv, const uint32_t (&nz)[16],
                                           float facc, const EscapeLog& log, CompressLds& S, uint64_t (&F)[16],
                                           uint64_t& myflag)
{
    uint32_t err = 0;
    if (__ballot(!(facc < 2147483648.0f))) {  // NaN, Inf or |x*inv| >= 2^31 somewhere in the layer
        err = classify_errors(x, scr, c, wave, inv, lane);
#pragma unroll
        for (int sh = 32; sh > 0; sh >>= 1) err |= (uint32_t)__shfl_xor((int)err, sh);
    }
    const int nout = log.count;

    // flags of the zero-block encoder: one ballot per bit plane
    uint32_t nnz = 0;
    myflag = 0;
#pragma unroll
    for (int b = 0; b < 16; b++) {
        F[b] = __ballot(nz[b] != 0u);
        nnz += __popcll(F[b]);
        myflag = lane == b ? F[b] : myflag;
    }
    if (lane == 0) {
        S.nnz[wave] = nnz;
        S.nout[wave] = (uint32_t)nout;
        if (err) atomicOr(&S.err, err);
        // the chunk's last wave to get here publishes its size at once: a
        // size published after the workgroup barrier would wait for this
        // workgroup's look-back, and other look-backs for it in turn
        if (__hip_atomic_fetch_add(&S.arrived, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == kLayers - 1) {
            S.arrived = 0;  // the next chunk's waves arrive after a barrier
            publish_state(reinterpret_cast<uint64_t*>(const_cast<uint8_t*>(scr) + kScratchStateOff) + c,
                          kFlagAgg | chunk_units(S));
        }
    }
    return nout;
}

// A layer of a chunk cut by the field's edge, after the fast pass: its
// cells outside the field were loaded as other chunks' values (or zeros past
// the field's end), so their codes are cleared in the layer's plane words in
// LDS (bit i of each word is code i of the lane's patch); the caller then
// gathers the flags' nonzero bits again.  Such a cell's delta may also have
// reported an escape; the layer has then taken the logging pass instead,
// which zeroes those deltas before it looks for escapes.  A real call, with
// plain arguments and LDS only: inlined, or with arrays passed to it, it
// pushes the fast path into spills.  The words are addressed as LDS (a plain
// pointer made them flat accesses, in 2-D each read waited for before its
// write), a step's 16 words read before any is written back.
typedef __attribute__((address_space(3))) uint32_t LdsWord;
template <int RANK>
__device__ __noinline__ void mask_layer(LdsWord* Wl, int64_t e0, int64_t e1, int64_t e2, uint32_t off, int k, int lane)
{
    Lane l;
    l.ext[0] = e0;
    l.ext[1] = e1;
    l.ext[2] = e2;
    l.off = off;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const uint32_t keep = keep_bits<RANK>(l, 4 * k + t, lane);
        uint32_t w[16];
#pragma unroll
        for (int b = 0; b < 16; b++) w[b] = Wl[(b * 4 + t) * 64 + lane];
#pragma unroll
        for (int b = 0; b < 16; b++) Wl[(b * 4 + t) * 64 + lane] = w[b] & keep;
    }
}

// Wave `wave`'s layer of chunk c: bricks into S.w[wave], its brick and
// escape counts into S.  `h` / `v` hold the prefetched halo and first step
// (the top two steps of a layer swept downwards).  F receives the layer's per-plane ballots and `myflag` the
// flag word lane b < 16 stores; returns the layer's escape count.
template <int RANK, bool VEC4, int QM = kQuantGrid>
__device__ __forceinline__ int chunk_layer(const float* __restrict__ x, const uint8_t* __restrict__ scr, const Geom& g,
                                           int64_t c, const Lane& l, int wave, int lane, Quant inv, float (&h)[32],
                                           float (&v)[32], CompressLds& S, uint64_t (&F)[16], uint64_t& myflag)
{
    uint32_t nz[16];
    float facc = 0.0f;
    uint32_t* Wl = S.w[wave];
    EscapeLog log{nullptr, 0, 0};
    if (wave < l.L) {
        bool slow;
        if constexpr (RANK >= 2) {
            slow = swept_down<RANK>(wave)
                       ? layer_rev<RANK, VEC4, QM>(x, g, l, wave, inv, lane, h, v, Wl, nz, facc, log)
                       : layer<RANK, VEC4, false, QM>(x, g, l, wave, inv, lane, h, v, Wl, nz, facc, log);
            if (!slow && l.edge)  // uniform: clear the codes of cells outside the field
                mask_layer<RANK>((LdsWord*)Wl, l.ext[0], l.ext[1], l.ext[2], l.off, wave, lane);
        } else {
            // 1-D: only a field's last chunk is cut by its edge; it takes the
            // logging pass, which masks the deltas itself (a mask call here
            // measured as spills in the 1-D fast path)
            slow = layer<RANK, VEC4, false, QM>(x, g, l, wave, inv, lane, h, v, Wl, nz, facc, log) || l.edge;
        }
        if (slow) {  // escapes to log
            const uint64_t r = layer_slow<RANK, VEC4, QM>(x, scr, c, wave, inv, lane, Wl, nullptr, 0);
            log.count = (int)(r >> 32);
            facc = __builtin_elementwise_maximum(facc, __uint_as_float((uint32_t)r));
        }
        if (slow || l.edge) {  // the layer's words were rewritten in LDS: their nonzero bits again
#pragma unroll
            for (int b = 0; b < 16; b++)
                nz[b] = Wl[(b * 4) * 64 + lane] | Wl[(b * 4 + 1) * 64 + lane] | Wl[(b * 4 + 2) * 64 + lane] |
                        Wl[(b * 4 + 3) * 64 + lane];
        }
    } else {
#pragma unroll
        for (int b = 0; b < 16; b++) nz[b] = 0u;
    }
    return layer_flags(x, scr, g, c, wave, lane, inv, nz, facc, log, S, F, myflag);
}

// polls of a look-back before it gives up (each poll sleeps about 64 cycles
// and waits for a load that bypasses the L2; far beyond any real wait)
constexpr int kLookbackSpins = 1 << 18;

// Exclusive prefix of chunk c's payload size (Sec. 3.4: the offset of its
// data blocks), by one wave: the published states of chunks c-1, c-2, ... are
// read 64 at a time and summed back to the nearest chunk that published its
// inclusive prefix.  Chunks that have not published their size yet are polled
// until they do (every chunk before c was taken by a running workgroup, which
// publishes its size without waiting for anything).  Returns false if the
// polls ran out (the stream is then marked with an internal error).
__device__ __forceinline__ bool lookback(const uint64_t* state, int64_t c, int lane, uint64_t& excl)
{
    uint64_t sum = 0;
    for (int64_t hi = c; hi > 0; hi -= 64) {
        const int64_t i = hi - 1 - lane;  // lane 0 reads the nearest chunk
        uint64_t v = i >= 0 ? peek_state(state + i) : kFlagIncl;  // before chunk 0: inclusive prefix 0
        for (int spin = 0;; spin++) {
            const uint64_t incl = __ballot((v & ~kValueMask) == kFlagIncl);
            const int first = incl ? __builtin_ctzll(incl) : 64;
            const uint64_t below = first == 64 ? ~0ull : (1ull << first) - 1;
            const uint64_t miss = __ballot((v & ~kValueMask) == 0) & below;
            if (!miss) {
                uint64_t t = lane <= first ? (v & kValueMask) : 0;
#pragma unroll
                for (int sh = 32; sh > 0; sh >>= 1) t += __shfl_xor(t, sh);
                sum += t;
                if (incl) {
                    excl = sum;
                    return true;
                }
                break;
            }
            if (spin >= kLookbackSpins) {
                excl = 0;
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
            if ((miss >> lane) & 1ull) v = peek_state(state + i);
        }
    }
    excl = sum;
    return true;
}

// After a workgroup barrier that follows chunk_layer on all 4 waves: the
// layer's flags go to the stream (stored only here, so that no wait before
// the barrier covers them), the chunk's escape count to the table, the counts
// to the header, and its payload is assembled in the workgroup's staging slot:
// nonzero bricks in (layer, plane, patch) order, then the escape pairs padded
// to 16 bytes.  A chunk may hold kChunkOutlierCap escapes wherever they fall;
// past that the stream carries the OUTLIER_CAP status and no pairs are
// written.  A layer with escapes is computed again out of line (its first
// pass kept only the count) and writes its pairs behind those of the layers
// before it.  The chunk's size was published by its last layer, before the
// barrier.
template <int RANK, bool VEC4, int QM = kQuantGrid>
__device__ __forceinline__ void stage_chunk(const float* __restrict__ x, uint8_t* __restrict__ out,
                                            const uint8_t* __restrict__ scr, const Geom& g,
                                            int64_t c, int wave, int lane, Quant inv, const uint64_t (&F)[16],
                                            uint64_t myflag, int nout, CompressLds& S, uint8_t* __restrict__ slot)
{
    if (lane < 16)
        reinterpret_cast<uint64_t*>(out + g.flags_off + (int64_t)kFlagBytesPerChunk * c + 128 * wave)[lane] = myflag;
    const uint32_t tn = S.nnz[0] + S.nnz[1] + S.nnz[2] + S.nnz[3];
    const uint32_t to = S.nout[0] + S.nout[1] + S.nout[2] + S.nout[3];
    const bool capped = to > (uint32_t)kChunkOutlierCap;
    const uint32_t kept = capped ? 0u : to;
    if (threadIdx.x == 0) {
        reinterpret_cast<uint32_t*>(out + g.table_off + 8 * c)[1] = kept;
        atomicAdd(reinterpret_cast<unsigned long long*>(out + kOffNnz), (unsigned long long)tn);
        atomicAdd(reinterpret_cast<unsigned long long*>(out + kOffNout), (unsigned long long)kept);
        const uint32_t err = S.err | (capped ? kErrOutlierCap : 0u);
        if (err) atomicOr(reinterpret_cast<uint32_t*>(out + kOffStatus), err);
        S.err = 0;
        if (kept & 1u) *reinterpret_cast<uint2*>(slot + 16 * tn + 8 * kept) = make_uint2(0u, 0u);
    }
    uint64_t base = 0;
    for (int w = 0; w < wave; w++) base += S.nnz[w];
    uint32_t* Wl = S.w[wave];
#pragma unroll
    for (int b = 0; b < 16; b++) {
        if (F[b] == 0) continue;  // uniform: a bit plane without nonzero bricks
        if ((F[b] >> lane) & 1ull) {
            const uint64_t pos = base + mbcnt(F[b]);
            const uint32_t* w = Wl + b * 4 * 64 + lane;
            *reinterpret_cast<uint4*>(slot + 16 * pos) = make_uint4(w[0], w[64], w[128], w[192]);
        }
        base += __popcll(F[b]);
    }
    if (nout && !capped) {  // rare: this layer's escape pairs, in code-index order
        uint32_t first = 0;
        for (int w = 0; w < wave; w++) first += S.nout[w];
        uint32_t* pairs = reinterpret_cast<uint32_t*>(slot + 16 * tn) + 2 * first;
        (void)layer_slow<RANK, VEC4, QM>(x, scr, c, wave, inv, lane, Wl, pairs, nout);
    }
}

// Placement of chunk p, staged in a workgroup's slot with `units` 16-B units
// of payload, in two parts.  place_lookback, by one wave (any time after the
// staging, before a barrier that precedes place_copy): the look-back finds
// the offset, thread 0 publishes the inclusive prefix, writes the offset to
// the table and, for the field's last chunk, the stream's total size to the
// header, and leaves the offset in S.excl.  A failed look-back marks the
// stream with an internal error and still publishes (as if at offset 0), so
// that no later chunk waits on this one; every offset stays inside the
// stream's bound.
__device__ __forceinline__ void place_lookback(uint8_t* __restrict__ out, uint8_t* __restrict__ scr, const Geom& g,
                                               int64_t p, uint32_t units, CompressLds& S, int lane)
{
    uint64_t* state = reinterpret_cast<uint64_t*>(scr + kScratchStateOff);
    uint64_t excl;
    const bool ok = lookback(state, p, lane, excl);
    if (lane == 0) {
        if (!ok) atomicOr(reinterpret_cast<uint32_t*>(out + kOffStatus), kErrInternal);
        const uint64_t at = ok ? excl : 0;
        S.excl = ok ? excl : ~0ull;
        publish_state(state + p, kFlagIncl | (at + units));
        reinterpret_cast<uint32_t*>(out + g.table_off)[2 * p] = (uint32_t)at;
        if (p == g.n_chunks - 1) *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off + 16 * (at + units);
    }
}

// place_copy, by the whole workgroup: the staged payload goes to its offset
// (read from the cache: the slot was written one chunk earlier).  Ends with a
// barrier, so the slot may be written again.
__device__ __forceinline__ void place_copy(uint8_t* __restrict__ out, const Geom& g, uint32_t units,
                                           const uint8_t* __restrict__ slot, const CompressLds& S)
{
    const uint64_t excl = S.excl;
    if (excl != ~0ull) {
        const uint4* src = reinterpret_cast<const uint4*>(slot);
        uint4* dst = reinterpret_cast<uint4*>(out + g.payload_off) + excl;
        for (uint32_t i = threadIdx.x; i < units; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
}

// ------------------------------------------------- per-field pipeline steps
// These bodies run for one field; the per-field kernels call them with the
// whole grid, the batched kernels with the blocks given to that field.

// Header, table padding, scratch and chunk states of one field, by `nthreads`
// threads numbered `tid`.
__device__ __forceinline__ void init_field(uint8_t* __restrict__ out, uint8_t* __restrict__ scratch, const Geom& g,
                                           const HeaderImage& h, int64_t tid,
                                           int64_t nthreads)
{
    if (tid < kHeaderBytes / 4) reinterpret_cast<uint32_t*>(out)[tid] = h.w[tid];
    if (tid == 0 && (g.n_chunks & 1))  // the chunk table is padded to 16 bytes with zeros
        *reinterpret_cast<uint2*>(out + g.table_off + 8 * g.n_chunks) = make_uint2(0u, 0u);
    uint32_t* scr = reinterpret_cast<uint32_t*>(scratch);
    if (tid < kScratchGeomOff / 4) scr[tid] = 0u;
    static_assert(sizeof(Geom) % 4 == 0 && kScratchGeomOff + sizeof(Geom) <= kScratchStateOff, "scratch layout");
    if (tid < (int64_t)(sizeof(Geom) / 4))
        scr[kScratchGeomOff / 4 + tid] = reinterpret_cast<const uint32_t*>(&g)[tid];
    uint64_t* state = reinterpret_cast<uint64_t*>(scratch + kScratchStateOff);
    for (int64_t i = tid; i < g.n_chunks; i += nthreads) state[i] = 0;
}

// Partial value range of block `blk` of `nblk` (256 threads each) for the
// relative error bound: the blocks walk the field from its end so that its
// beginning, which compression reads first, is the most recently touched
// data.  The partial (min key, max key, non-finite) goes to the scratch.
__device__ __forceinline__ void minmax_block(const float* __restrict__ x, int64_t n, uint8_t* __restrict__ scr,
                                             const Geom& g, int64_t blk, int64_t nblk)
{
    __shared__ uint32_t s_red[3][4];
    // NaN-propagating minimum / maximum over the raw values: the range is only
    // used when every value is finite, and a NaN or an infinity shows up in
    // the result (the minimum is -Inf or NaN, or the maximum +Inf or NaN)
    float fmn = __builtin_inff(), fmx = -__builtin_inff();
    auto take4 = [&](const fz_f32x4& v) {
        fmn = __builtin_elementwise_minimum(__builtin_elementwise_minimum(fmn, v.x), v.y);
        fmx = __builtin_elementwise_maximum(__builtin_elementwise_maximum(fmx, v.x), v.y);
        fmn = __builtin_elementwise_minimum(__builtin_elementwise_minimum(fmn, v.z), v.w);
        fmx = __builtin_elementwise_maximum(__builtin_elementwise_maximum(fmx, v.z), v.w);
    };
    const int64_t stride = nblk * 256;
    const int64_t tid = blk * 256 + threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    const fz_f32x4* x4 = reinterpret_cast<const fz_f32x4*>(x);
    // backwards, so that the front of the field, which the compression
    // kernel reads first, is the most recently read (one load per
    // iteration: unrolling by strided loads measured slower); streaming
    // loads, as no value is read twice here
    for (int64_t i = n4 - 1 - tid; i >= 0; i -= stride) take4(__builtin_nontemporal_load(x4 + i));
    for (int64_t k = 4 * n4 + tid; k < n; k += stride) {
        fmn = __builtin_elementwise_minimum(fmn, x[k]);
        fmx = __builtin_elementwise_maximum(fmx, x[k]);
    }
    const bool some = fmn <= fmx;  // false for a thread without values (and for NaN)
    uint32_t bad = (fmn >= -3.40282347e38f && fmx <= 3.40282347e38f) ? 0u : 1u;
    uint32_t lo = some ? float_key(fmn) : 0xFFFFFFFFu, hi = some ? float_key(fmx) : 0u;
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, sh));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, sh));
        bad |= (uint32_t)__shfl_xor((int)bad, sh);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_red[0][w] = lo; s_red[1][w] = hi; s_red[2][w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* part = reinterpret_cast<uint32_t*>(scr + g.scr_minmax) + 4 * blk;
        part[0] = min(min(s_red[0][0], s_red[0][1]), min(s_red[0][2], s_red[0][3]));
        part[1] = max(max(s_red[1][0], s_red[1][1]), max(s_red[1][2], s_red[1][3]));
        part[2] = s_red[2][0] | s_red[2][1] | s_red[2][2] | s_red[2][3];
    }
}

// The eb parameters of a REL compression, from the folded value range.
struct RelParams {
    uint32_t status;          // 0, kErrNonfinite or kErrEbRange
    float ebx2, inv, vmin, vmax;
};

// Fold the partial ranges of one field and derive the eb parameters, by one
// block of blockDim.x threads (a multiple of 64, at most 1024); every thread
// gets the result.  eb_abs = eb * (vmax - vmin) in double (a constant field
// uses eb * |vmax|, or eb if that is 0), ebx2 = fp32(2 eb_abs),
// inv = fp32(1 / (double)ebx2).
__device__ __forceinline__ RelParams fold_params(const uint8_t* __restrict__ scratch, const Geom& g, double eb,
                                                 int nparts)
{
    __shared__ uint32_t s_red[3][16];
    // the partials (16 B each) in 16-byte loads, 8 per thread in flight
    // together: every compression workgroup folds them before its first
    // chunk, and one load at a time cost a cache round trip per 256 partials
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(scratch + g.scr_minmax), (short)0, 16 * nparts, kBufferFlags);
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, bad = 0u;
    for (int i0 = 0; i0 < nparts; i0 += 8 * (int)blockDim.x) {
        fz_u32x4 t[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            t[k] = __builtin_amdgcn_raw_buffer_load_b128(rp, 16u * (uint32_t)(i0 + k * blockDim.x + threadIdx.x), 0u, 0);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (i0 + k * (int)blockDim.x + (int)threadIdx.x < nparts) {
                lo = min(lo, t[k].x);
                hi = max(hi, t[k].y);
                bad |= t[k].z;
            }
        }
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, sh));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, sh));
        bad |= (uint32_t)__shfl_xor((int)bad, sh);
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_red[0][w] = lo; s_red[1][w] = hi; s_red[2][w] = bad; }
    __syncthreads();
    lo = 0xFFFFFFFFu, hi = 0u, bad = 0u;
    for (int i = 0; i < nw; i++) {
        lo = min(lo, s_red[0][i]);
        hi = max(hi, s_red[1][i]);
        bad |= s_red[2][i];
    }
    // the same on every lane: kept scalar, so that a branch on the result is
    // uniform and nothing after it is treated as divergent
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    bad = __builtin_amdgcn_readfirstlane(bad);
    __syncthreads();  // s_red may be reused by the caller's next fold
    RelParams r{0u, 0.0f, 0.0f, 0.0f, 0.0f};
    if (bad) {
        r.status = kErrNonfinite;
    } else {
        r.vmin = key_float(lo);
        r.vmax = key_float(hi);
        const double range = (double)r.vmax - (double)r.vmin;
        double eb_abs;
        if (range > 0.0) eb_abs = eb * range;
        else {
            const double a = __builtin_fabs((double)r.vmax);
            eb_abs = eb * (a > 0.0 ? a : 1.0);
        }
        r.ebx2 = (float)(2.0 * eb_abs);
        r.inv = (float)(1.0 / (double)r.ebx2);
        if (!(r.ebx2 >= 1.17549435e-38f) || !__builtin_isfinite(r.ebx2) || !__builtin_isfinite(r.inv) || !(r.inv > 0.0f))
            r.status = kErrEbRange;
    }
    return r;
}

// The header's eb fields (and, on a failed range, its status and total) and
// the scratch's pre_status, by one thread.
__device__ __forceinline__ void write_params(uint8_t* __restrict__ out, uint8_t* __restrict__ scratch, const Geom& g,
                                             const RelParams& r)
{
    *reinterpret_cast<float*>(out + kOffEbx2) = r.ebx2;
    *reinterpret_cast<float*>(out + kOffInv) = r.inv;
    *reinterpret_cast<float*>(out + kOffVmin) = r.vmin;
    *reinterpret_cast<float*>(out + kOffVmax) = r.vmax;
    if (r.status) {
        *reinterpret_cast<uint32_t*>(out + kOffStatus) = r.status;
        *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off;
    }
    reinterpret_cast<Scratch*>(scratch)->pre_status = r.status;
}

// The eb parameters by a block of its own (the batch layer, the field-global
// predictor): fold, then thread 0 writes them.
__device__ __forceinline__ void params_field(uint8_t* __restrict__ out, uint8_t* __restrict__ scratch, const Geom& g,
                                             double eb, int nparts)
{
    const RelParams r = fold_params(scratch, g, eb, nparts);
    if (threadIdx.x == 0) write_params(out, scratch, g, r);
}

// End of one field's compression, after every chunk is placed (a launch of
// its own): a failed prequantization anywhere (NaN/Inf, overflow) ends the
// pipeline before the encoder, so the escape-cap bit of chunks that went on
// counts only when no such bit is set.
__device__ __forceinline__ void finish_field(uint8_t* __restrict__ out, const uint8_t* __restrict__ scratch)
{
    const Scratch* scr = reinterpret_cast<const Scratch*>(scratch);
    if (scr->pre_status) return;  // the range pass failed: nothing was compressed
    uint32_t* st = reinterpret_cast<uint32_t*>(out + kOffStatus);
    const uint32_t v = *st;
    if (v & (kErrNonfinite | kErrEbRange)) *st = v & ~kErrOutlierCap;
}

// The same inside the per-field compression kernel, by thread 0 of each
// workgroup as it ends (after its last placement and barrier): the last
// workgroup of the grid to count itself done settles the status word, so
// that no launch of its own is needed.  The status word and the count are
// only touched with agent-scope atomics, which every XCD sees in one order
// (their L2 caches are not coherent with one another, so nothing here may
// rely on them).  Thread 0 set its workgroup's status bits; an explicit wait
// for its outstanding memory operations (not an agent-scope release, which
// adds an L2 write-back at every workgroup's end: +9 us on 512^3) makes those
// atomics complete before the count is issued, and the last workgroup
// reads and clears the word only after its count has returned.  Workgroups
// that return because the range pass failed (pre_status) do not count;
// nothing is settled then.
__device__ __forceinline__ void finish_if_last(uint8_t* __restrict__ out, uint8_t* __restrict__ scratch)
{
    if (threadIdx.x != 0) return;
    Scratch* scr = reinterpret_cast<Scratch*>(scratch);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // no memory operation moves below this point
    __builtin_amdgcn_s_waitcnt(0);  // and every one of this thread's has completed (the fence alone emits no wait)
    if (__hip_atomic_fetch_add(&scr->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gridDim.x - 1) return;
    uint32_t* st = reinterpret_cast<uint32_t*>(out + kOffStatus);
    const uint32_t v = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v & (kErrNonfinite | kErrEbRange))
        __hip_atomic_fetch_and(st, ~kErrOutlierCap, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace fz
