// fz_compress.hip -- single-pass compression kernel of libfzmi (gfx950).
//
// One workgroup (4 waves) per chunk, one wave per layer of 4 steps, one lane
// per 32-code patch.  Per step a lane: loads its 32 fp32 values, prequantizes
// them (Sec. 2.3), applies the Lorenzo difference on the integers (Sec. 2.3 /
// 3.2; the previous step sits in the same lane's registers, the other two
// neighbours come from adjacent lanes), maps them to sign-magnitude 16-bit
// codes (Sec. 3.2), and bit-transposes the 32 codes in registers (Sec. 3.3).
// After its 4 steps a lane holds 16 bricks (one per bit plane); a ballot per
// plane gives the bit flags of the zero-block encoder (Sec. 3.4).  The
// workgroup then takes its payload offset from a decoupled look-back over
// the preceding chunks (the device-wide exclusive prefix sum of Sec. 3.4,
// here without a second kernel) and every lane stores its nonzero bricks
// with coalesced 16-byte writes.  No intermediate array touches HBM.
#include <hip/hip_runtime.h>

#include "fz_device.hpp"
#include "fz_kernels.hpp"

namespace fz {

struct EscapeLog {
    uint32_t* idx;  // LDS, kLayerOutlierCap entries for this wave
    int32_t* val;
    int count;      // escapes seen so far in this layer (may exceed the cap)
};

// Slow path of a step with at least one escape: codes whose delta does not
// fit in 15 bits become 0x8000 and their (code index, delta) pair is logged
// in code-index order (lane-major, then cell).
__device__ __forceinline__ void log_escapes(const int (&d)[32], uint32_t (&P)[16], EscapeLog& log, uint32_t n0, int lane)
{
    uint32_t emask = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) emask |= (absu(d[i]) > 32767u ? 1u : 0u) << i;
    const int cnt = __popc(emask);
    const int incl = wave_incl_scan(cnt, lane);
    const int total = __shfl(incl, 63);
    int pos = log.count + incl - cnt;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if ((emask >> i) & 1u) {
            if (pos < kLayerOutlierCap) {
                log.idx[pos] = n0 + (uint32_t)lane * kPatchCodes + i;
                log.val[pos] = d[i];
            }
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

// codes -> escapes -> bit planes, shared tail of every rank's step
__device__ __forceinline__ void finish_step(const int (&d)[32], uint32_t (&P)[16], EscapeLog& log, uint32_t n0, int lane)
{
    uint32_t macc = 0;
    pack_codes(d, P, macc);
    if (__ballot(macc > 32767u)) log_escapes(d, P, log, n0, lane);
    transpose16(P);
}

// ------------------------------------------------------------------ loaders
template <int CNT, bool VEC4>
__device__ __forceinline__ void load_run(const float* __restrict__ p, float* v)
{
    if (VEC4) {
#pragma unroll
        for (int j = 0; j < CNT / 4; j++) {
            float4 t = *reinterpret_cast<const float4*>(p + 4 * j);
            v[4 * j] = t.x; v[4 * j + 1] = t.y; v[4 * j + 2] = t.z; v[4 * j + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < CNT; j++) v[j] = p[j];
    }
}

template <int CNT>
__device__ __forceinline__ void load_run_masked(const float* __restrict__ p, float* v, int valid)
{
#pragma unroll
    for (int j = 0; j < CNT; j++) v[j] = j < valid ? p[j] : 0.0f;
}

// ------------------------------------------------------------------- 3-D
// patch: rows y0..y0+3 (ey valid), cols x0..x0+7 (ex valid) of plane z
template <bool EDGE, bool VEC4>
__device__ __forceinline__ void load3(const float* __restrict__ x, const Geom& g, int64_t z, int64_t y0, int64_t x0,
                                      int ey, int ex, float (&v)[32])
{
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const float* p = x + ((z * g.n[1] + y0 + r) * g.n[2] + x0);
        if (EDGE) {
            if (r < ey) load_run_masked<8>(p, v + 8 * r, ex);
            else
#pragma unroll
                for (int j = 0; j < 8; j++) v[8 * r + j] = 0.0f;
        } else {
            load_run<8, VEC4>(p, v + 8 * r);
        }
    }
}

template <bool EDGE, bool VEC4>
__device__ __forceinline__ void layer3(const float* __restrict__ x, const Geom& g, const int64_t (&org)[3],
                                       const int64_t (&ext)[3], int k, float inv, int lane, uint32_t (&W)[16][4],
                                       uint32_t& facc, EscapeLog& log)
{
    const int py = lane & 7, px = lane >> 3;
    const int64_t y0 = org[1] + 4 * py, x0 = org[2] + 8 * px;
    const int ey = EDGE ? clampi(ext[1] - 4 * py, 0, 4) : 4;
    const int ex = EDGE ? clampi(ext[2] - 8 * px, 0, 8) : 8;
    int qprev[32];
    if (k == 0) {
#pragma unroll
        for (int i = 0; i < 32; i++) qprev[i] = 0;
    } else {  // halo: the plane just before this layer, same chunk
        float h[32];
        load3<EDGE, VEC4>(x, g, org[0] + 4 * k - 1, y0, x0, ey, ex, h);
#pragma unroll
        for (int i = 0; i < 32; i++) qprev[i] = prequant(h[i], inv, facc);
    }
    float v[32];
    load3<EDGE, VEC4>(x, g, org[0] + 4 * k, y0, x0, ey, ex, v);
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int s = 4 * k + t;
        if (s >= ext[0]) {
#pragma unroll
            for (int b = 0; b < 16; b++) W[b][t] = 0u;
            continue;
        }
        float vn[32];
        if (t < 3 && s + 1 < ext[0]) load3<EDGE, VEC4>(x, g, org[0] + s + 1, y0, x0, ey, ex, vn);
        int a[32];
#pragma unroll
        for (int i = 0; i < 32; i++) {
            const int q = prequant(v[i], inv, facc);
            a[i] = q - qprev[i];  // Dz
            qprev[i] = q;
        }
        int b[32];
#pragma unroll
        for (int c = 0; c < 8; c++) b[c] = a[c] - shift_up1(py == 7 ? 0 : a[24 + c], lane);  // Dy, row above from lane-1
#pragma unroll
        for (int r = 1; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 8; c++) b[8 * r + c] = a[8 * r + c] - a[8 * (r - 1) + c];
        int d[32];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int left = lane_value(b[8 * r + 7], lane - 8);  // Dx, column to the left from lane-8
            d[8 * r] = b[8 * r] - (px == 0 ? 0 : left);
#pragma unroll
            for (int c = 1; c < 8; c++) d[8 * r + c] = b[8 * r + c] - b[8 * r + c - 1];
        }
        if (EDGE) {
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int c = 0; c < 8; c++)
                    if (!(r < ey && c < ex)) d[8 * r + c] = 0;
        }
        uint32_t P[16];
        finish_step(d, P, log, (uint32_t)s * kStepCodes, lane);
#pragma unroll
        for (int bb = 0; bb < 16; bb++) W[bb][t] = P[bb];
#pragma unroll
        for (int i = 0; i < 32; i++) v[i] = vn[i];
    }
}

// ------------------------------------------------------------------- 2-D
template <bool EDGE, bool VEC4>
__device__ __forceinline__ void load2(const float* __restrict__ x, const Geom& g, int64_t y, int64_t x0, int ry, int ex,
                                      float* v)
{
    // one row of 16 values; ry = 1 if the row is inside the field
    const float* p = x + (y * g.n[1] + x0);
    if (EDGE) {
        if (ry) load_run_masked<16>(p, v, ex);
        else
#pragma unroll
            for (int j = 0; j < 16; j++) v[j] = 0.0f;
    } else {
        load_run<16, VEC4>(p, v);
    }
}

template <bool EDGE, bool VEC4>
__device__ __forceinline__ void layer2(const float* __restrict__ x, const Geom& g, const int64_t (&org)[3],
                                       const int64_t (&ext)[3], int k, float inv, int lane, uint32_t (&W)[16][4],
                                       uint32_t& facc, EscapeLog& log)
{
    const int64_t x0 = org[1] + 16 * lane;
    const int ex = EDGE ? clampi(ext[1] - 16 * lane, 0, 16) : 16;
    int qprev[16];
    if (k == 0) {
#pragma unroll
        for (int i = 0; i < 16; i++) qprev[i] = 0;
    } else {  // halo: the row just before this layer
        float h[16];
        load2<EDGE, VEC4>(x, g, org[0] + 8 * k - 1, x0, 1, ex, h);
#pragma unroll
        for (int i = 0; i < 16; i++) qprev[i] = prequant(h[i], inv, facc);
    }
    float v[32];
    {
        const int64_t yr = 8 * k;
        load2<EDGE, VEC4>(x, g, org[0] + yr, x0, yr < ext[0], ex, v);
        load2<EDGE, VEC4>(x, g, org[0] + yr + 1, x0, yr + 1 < ext[0], ex, v + 16);
    }
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int s = 4 * k + t;
        if (2 * s >= ext[0]) {
#pragma unroll
            for (int b = 0; b < 16; b++) W[b][t] = 0u;
            continue;
        }
        float vn[32];
        if (t < 3 && 2 * (s + 1) < ext[0]) {
            load2<EDGE, VEC4>(x, g, org[0] + 2 * (s + 1), x0, 1, ex, vn);
            load2<EDGE, VEC4>(x, g, org[0] + 2 * (s + 1) + 1, x0, 2 * (s + 1) + 1 < ext[0], ex, vn + 16);
        }
        int q[32];
#pragma unroll
        for (int i = 0; i < 32; i++) q[i] = prequant(v[i], inv, facc);
        int b[32];
#pragma unroll
        for (int c = 0; c < 16; c++) {
            b[c] = q[c] - qprev[c];          // Dy against the previous row (same lane)
            b[16 + c] = q[16 + c] - q[c];
            qprev[c] = q[16 + c];
        }
        int d[32];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            d[16 * r] = b[16 * r] - shift_up1(b[16 * r + 15], lane);  // Dx, left column from lane-1 (0 at lane 0)
#pragma unroll
            for (int c = 1; c < 16; c++) d[16 * r + c] = b[16 * r + c] - b[16 * r + c - 1];
        }
        if (EDGE) {
            const bool r1 = 2 * s + 1 < ext[0];
#pragma unroll
            for (int c = 0; c < 16; c++) {
                if (!(c < ex)) d[c] = 0;
                if (!(c < ex && r1)) d[16 + c] = 0;
            }
        }
        uint32_t P[16];
        finish_step(d, P, log, (uint32_t)s * kStepCodes, lane);
#pragma unroll
        for (int bb = 0; bb < 16; bb++) W[bb][t] = P[bb];
#pragma unroll
        for (int i = 0; i < 32; i++) v[i] = vn[i];
    }
}

// ------------------------------------------------------------------- 1-D
template <bool EDGE, bool VEC4>
__device__ __forceinline__ void layer1(const float* __restrict__ x, const Geom& g, const int64_t (&org)[3],
                                       const int64_t (&ext)[3], int k, float inv, int lane, uint32_t (&W)[16][4],
                                       uint32_t& facc, EscapeLog& log)
{
    int carry = 0;  // q just before the current step (uniform)
    if (k > 0) {
        uint32_t dummy = 0;
        carry = prequant(x[org[0] + 8192 * k - 1], inv, dummy);
    }
    auto valid_of = [&](int s) -> int {
        return EDGE ? clampi(ext[0] - ((int64_t)kStepCodes * s + kPatchCodes * lane), 0, 32) : 32;
    };
    float v[32];
    {
        const int s = 4 * k;
        const float* p = x + org[0] + (int64_t)kStepCodes * s + kPatchCodes * lane;
        if (EDGE) load_run_masked<32>(p, v, valid_of(s));
        else load_run<32, VEC4>(p, v);
    }
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int s = 4 * k + t;
        if ((int64_t)kStepCodes * s >= ext[0]) {
#pragma unroll
            for (int b = 0; b < 16; b++) W[b][t] = 0u;
            continue;
        }
        float vn[32];
        if (t < 3 && (int64_t)kStepCodes * (s + 1) < ext[0]) {
            const float* p = x + org[0] + (int64_t)kStepCodes * (s + 1) + kPatchCodes * lane;
            if (EDGE) load_run_masked<32>(p, vn, valid_of(s + 1));
            else load_run<32, VEC4>(p, vn);
        }
        int q[32];
#pragma unroll
        for (int i = 0; i < 32; i++) q[i] = prequant(v[i], inv, facc);
        int d[32];
        const int left = shift_up1(q[31], lane);
        d[0] = q[0] - (lane == 0 ? carry : left);
#pragma unroll
        for (int m = 1; m < 32; m++) d[m] = q[m] - q[m - 1];
        carry = __builtin_amdgcn_readlane(q[31], 63);
        if (EDGE) {
            const int valid = valid_of(s);
#pragma unroll
            for (int m = 0; m < 32; m++)
                if (!(m < valid)) d[m] = 0;
        }
        uint32_t P[16];
        finish_step(d, P, log, (uint32_t)s * kStepCodes, lane);
#pragma unroll
        for (int bb = 0; bb < 16; bb++) W[bb][t] = P[bb];
#pragma unroll
        for (int i = 0; i < 32; i++) v[i] = vn[i];
    }
}

// Rare path: a step saw NaN/Inf or |x*inv| >= 2^31.  Re-read the layer's
// cells and classify them the way the format defines the status bits.
__device__ __forceinline__ uint32_t classify_errors(const float* __restrict__ x, const Geom& g, const int64_t (&org)[3],
                                                 const int64_t (&ext)[3], int k, float inv, int lane)
{
    uint32_t err = 0;
    for (int t = 0; t < 4; t++) {
        const int s = 4 * k + t;
        for (int m = 0; m < 32; m++) {
            int64_t r[3] = {0, 0, 0};
            if (g.rank == 3) { r[0] = s; r[1] = 4 * (lane % 8) + m / 8; r[2] = 8 * (lane / 8) + m % 8; }
            else if (g.rank == 2) { r[0] = 2 * s + m / 16; r[1] = 16 * lane + m % 16; }
            else { r[0] = (int64_t)kStepCodes * s + kPatchCodes * lane + m; }
            if (r[0] >= ext[0] || r[1] >= ext[1] || r[2] >= ext[2]) continue;
            const float v = x[((org[0] + r[0]) * g.n[1] + org[1] + r[1]) * g.n[2] + org[2] + r[2]];
            if (!__builtin_isfinite(v)) err |= kErrNonfinite;
            else if (!(__builtin_fabsf(v * inv) < 2147483648.0f)) err |= kErrEbRange;
        }
    }
    return err;  // halo values belong to the previous layer, which reports them
}

// Decoupled look-back (single-pass exclusive prefix sum over chunks): publish
// this chunk's aggregate, walk back accumulating aggregates until a chunk with
// a published inclusive prefix, then publish ours.  Tickets are taken in
// order, so every chunk waited on has a running or finished workgroup.
__device__ uint64_t lookback(uint64_t* state, int64_t c, uint64_t agg)
{
    if (c == 0) {
        __hip_atomic_store(&state[0], kFlagIncl | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    __hip_atomic_store(&state[c], kFlagAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t j = c - 1;
    for (;;) {
        const uint64_t v = __hip_atomic_load(&state[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t f = v & ~kValueMask;
        if (f == 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += v & kValueMask;
        if (f == kFlagIncl) break;
        j--;
    }
    __hip_atomic_store(&state[c], kFlagIncl | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

template <int RANK, bool EDGE, bool VEC4>
__device__ __forceinline__ void run_layer(const float* __restrict__ x, const Geom& g, const int64_t (&org)[3],
                                          const int64_t (&ext)[3], int k, float inv, int lane, uint32_t (&W)[16][4],
                                          uint32_t& facc, EscapeLog& log)
{
    if (RANK == 3) layer3<EDGE, VEC4>(x, g, org, ext, k, inv, lane, W, facc, log);
    else if (RANK == 2) layer2<EDGE, VEC4>(x, g, org, ext, k, inv, lane, W, facc, log);
    else layer1<EDGE, VEC4>(x, g, org, ext, k, inv, lane, W, facc, log);
}

template <int RANK, bool VEC4>
__global__ __launch_bounds__(256, 2) void k_compress(const float* __restrict__ x, uint8_t* __restrict__ out, Geom g)
{
    __shared__ uint32_t s_chunk, s_err;
    __shared__ uint32_t s_nnz[kLayers], s_nout[kLayers];
    __shared__ uint64_t s_off;
    __shared__ uint32_t s_oidx[kLayers][kLayerOutlierCap];
    __shared__ int32_t s_oval[kLayers][kLayerOutlierCap];

    Scratch* scr = reinterpret_cast<Scratch*>(out + g.scratch_off);
    uint64_t* state = reinterpret_cast<uint64_t*>(out + g.scratch_off + kScratchStateOff);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (scr->pre_status) return;  // set before this launch: uniform across the grid

    if (threadIdx.x == 0) {
        s_chunk = atomicAdd(&scr->ticket, 1u);
        s_err = 0;
    }
    __syncthreads();
    const int64_t c = s_chunk;
    const float inv = *reinterpret_cast<const float*>(out + kOffInv);
    int64_t org[3], ext[3];
    chunk_box(g, c, org, ext);
    const int L = layers_of(RANK, ext[0]);
    bool edge = false;
#pragma unroll
    for (int i = 0; i < 3; i++) edge |= ext[i] < g.box[i];

    uint32_t W[16][4];
    uint32_t facc = 0;
    EscapeLog log{s_oidx[wave], s_oval[wave], 0};
    if (wave < L) {
        if (edge) run_layer<RANK, true, VEC4>(x, g, org, ext, wave, inv, lane, W, facc, log);
        else run_layer<RANK, false, VEC4>(x, g, org, ext, wave, inv, lane, W, facc, log);
    } else {
#pragma unroll
        for (int b = 0; b < 16; b++)
#pragma unroll
            for (int t = 0; t < 4; t++) W[b][t] = 0u;
    }
    uint32_t err = 0;
    if (__ballot(facc >= kPrequantLimit)) {
        err = classify_errors(x, g, org, ext, wave, inv, lane);
#pragma unroll
        for (int sh = 32; sh > 0; sh >>= 1) err |= (uint32_t)__shfl_xor((int)err, sh);
    }
    if (log.count > kLayerOutlierCap) err |= kErrOutlierCap;
    const int nout = log.count < kLayerOutlierCap ? log.count : kLayerOutlierCap;

    // flags of the zero-block encoder: one ballot per bit plane
    uint64_t F[16];
    uint32_t nnz = 0;
    uint64_t myflag = 0;
#pragma unroll
    for (int b = 0; b < 16; b++) {
        F[b] = __ballot((W[b][0] | W[b][1] | W[b][2] | W[b][3]) != 0u);
        nnz += __popcll(F[b]);
        myflag = lane == b ? F[b] : myflag;
    }
    if (lane < 16)
        reinterpret_cast<uint64_t*>(out + g.flags_off + (int64_t)kFlagBytesPerChunk * c + 128 * wave)[lane] = myflag;
    if (lane == 0) {
        s_nnz[wave] = nnz;
        s_nout[wave] = (uint32_t)nout;
        if (err) atomicOr(&s_err, err);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tn = s_nnz[0] + s_nnz[1] + s_nnz[2] + s_nnz[3];
        const uint32_t to = s_nout[0] + s_nout[1] + s_nout[2] + s_nout[3];
        const uint64_t units = tn + (to + 1) / 2;
        const uint64_t excl = lookback(state, c, units);
        s_off = excl;
        uint32_t* tab = reinterpret_cast<uint32_t*>(out + g.table_off + 8 * c);
        tab[0] = (uint32_t)excl;
        tab[1] = to;
        atomicAdd(reinterpret_cast<unsigned long long*>(out + kOffNnz), (unsigned long long)tn);
        atomicAdd(reinterpret_cast<unsigned long long*>(out + kOffNout), (unsigned long long)to);
        if (s_err) atomicOr(reinterpret_cast<uint32_t*>(out + kOffStatus), s_err);
        if (c == g.n_chunks - 1)
            *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off + 16 * (excl + units);
        // payload is followed by the chunk's escape pairs, padded to 16 B
        if (to & 1u) {
            uint8_t* pairs = out + g.payload_off + 16 * (excl + tn);
            *reinterpret_cast<uint2*>(pairs + 8 * to) = make_uint2(0u, 0u);
        }
    }
    __syncthreads();

    // compaction: nonzero bricks in (layer, plane, patch) order
    uint64_t base = s_off;
    for (int w = 0; w < wave; w++) base += s_nnz[w];
    uint8_t* pay = out + g.payload_off;
#pragma unroll
    for (int b = 0; b < 16; b++) {
        if ((F[b] >> lane) & 1ull) {
            const uint64_t pos = base + mbcnt(F[b]);
            *reinterpret_cast<uint4*>(pay + 16 * pos) = make_uint4(W[b][0], W[b][1], W[b][2], W[b][3]);
        }
        base += __popcll(F[b]);
    }
    if (nout) {
        const uint32_t tn = s_nnz[0] + s_nnz[1] + s_nnz[2] + s_nnz[3];
        uint32_t first = 0;
        for (int w = 0; w < wave; w++) first += s_nout[w];
        uint32_t* pairs = reinterpret_cast<uint32_t*>(pay + 16 * (s_off + tn));
        for (int i = lane; i < nout; i += 64) {
            pairs[2 * (first + i)] = s_oidx[wave][i];
            pairs[2 * (first + i) + 1] = (uint32_t)s_oval[wave][i];
        }
    }
}

// ----------------------------------------------------------- setup kernels
__global__ void k_init(uint8_t* __restrict__ out, Geom g, HeaderImage h)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kHeaderBytes / 4) reinterpret_cast<uint32_t*>(out)[tid] = h.w[tid];
    if (tid == 0 && (g.n_chunks & 1))  // the chunk table is padded to 16 bytes with zeros
        *reinterpret_cast<uint2*>(out + g.table_off + 8 * g.n_chunks) = make_uint2(0u, 0u);
    uint32_t* scr = reinterpret_cast<uint32_t*>(out + g.scratch_off);
    if (tid < kScratchStateOff / 4) {
        uint32_t v = 0;
        if (tid == 2) v = 0xFFFFFFFFu;  // min_key
        scr[tid] = v;
    }
    uint64_t* state = reinterpret_cast<uint64_t*>(out + g.scratch_off + kScratchStateOff);
    for (int64_t i = tid; i < g.n_chunks; i += (int64_t)gridDim.x * blockDim.x) state[i] = 0;
}

__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ x, int64_t n, uint8_t* __restrict__ out,
                                                Geom g)
{
    Scratch* scr = reinterpret_cast<Scratch*>(out + g.scratch_off);
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, bad = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    // walk from the end so that the first chunks are the most recently read
    for (int64_t i = n4 - 1 - tid; i >= 0; i -= stride) {
        const float4 v = reinterpret_cast<const float4*>(x)[i];
        const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (!__builtin_isfinite(e[j])) { bad = 1u; continue; }
            const uint32_t key = float_key(e[j]);
            lo = min(lo, key);
            hi = max(hi, key);
        }
    }
    for (int64_t i = 4 * n4 + tid; i < n; i += stride) {
        const float e = x[i];
        if (!__builtin_isfinite(e)) { bad = 1u; continue; }
        const uint32_t key = float_key(e);
        lo = min(lo, key);
        hi = max(hi, key);
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, sh));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, sh));
        bad |= (uint32_t)__shfl_xor((int)bad, sh);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&scr->min_key, lo);
        atomicMax(&scr->max_key, hi);
        if (bad) atomicOr(&scr->nonfinite, 1u);
    }
}

__global__ void k_params(uint8_t* __restrict__ out, Geom g, double eb)
{
    Scratch* scr = reinterpret_cast<Scratch*>(out + g.scratch_off);
    uint32_t status = 0;
    float e2 = 0.0f, iv = 0.0f, lo = 0.0f, hi = 0.0f;
    if (scr->nonfinite) {
        status = kErrNonfinite;
    } else {
        lo = key_float(scr->min_key);
        hi = key_float(scr->max_key);
        const double range = (double)hi - (double)lo;
        double eb_abs;
        if (range > 0.0) eb_abs = eb * range;
        else {
            const double a = __builtin_fabs((double)hi);
            eb_abs = eb * (a > 0.0 ? a : 1.0);
        }
        e2 = (float)(2.0 * eb_abs);
        iv = (float)(1.0 / (double)e2);
        if (!(e2 >= 1.17549435e-38f) || !__builtin_isfinite(e2) || !__builtin_isfinite(iv) || !(iv > 0.0f))
            status = kErrEbRange;
    }
    *reinterpret_cast<float*>(out + kOffEbx2) = e2;
    *reinterpret_cast<float*>(out + kOffInv) = iv;
    *reinterpret_cast<float*>(out + kOffVmin) = lo;
    *reinterpret_cast<float*>(out + kOffVmax) = hi;
    if (status) {
        *reinterpret_cast<uint32_t*>(out + kOffStatus) = status;
        *reinterpret_cast<uint64_t*>(out + kOffTotal) = (uint64_t)g.payload_off;
    }
    scr->pre_status = status;
}

// ----------------------------------------------------------------- launch
template <int RANK, bool VEC4>
static hipError_t launch_rank(const float* x, uint8_t* out, const Geom& g, hipStream_t st)
{
    hipLaunchKernelGGL((k_compress<RANK, VEC4>), dim3((unsigned)g.n_chunks), dim3(256), 0, st, x, out, g);
    return hipGetLastError();
}

hipError_t launch_compress(const float* x, uint8_t* out, const Geom& g, const HeaderImage& h, bool rel, double eb,
                           hipStream_t st)
{
    const int64_t init_threads = g.n_chunks > kHeaderBytes / 4 ? g.n_chunks : kHeaderBytes / 4;
    const unsigned init_blocks = (unsigned)((init_threads + 255) / 256 < 1024 ? (init_threads + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_init, dim3(init_blocks), dim3(256), 0, st, out, g, h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (rel) {
        const int64_t n = g.n[0] * g.n[1] * g.n[2];
        int64_t blocks = (n / 4 + 255) / 256;
        if (blocks > 2048) blocks = 2048;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_minmax, dim3((unsigned)blocks), dim3(256), 0, st, x, n, out, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_params, dim3(1), dim3(1), 0, st, out, g, eb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const bool vec4 = (reinterpret_cast<uintptr_t>(x) & 15) == 0 && (g.rank == 1 || (g.n[g.rank - 1] & 3) == 0);
    switch (g.rank * 2 + (vec4 ? 1 : 0)) {
        case 7: return launch_rank<3, true>(x, out, g, st);
        case 6: return launch_rank<3, false>(x, out, g, st);
        case 5: return launch_rank<2, true>(x, out, g, st);
        case 4: return launch_rank<2, false>(x, out, g, st);
        case 3: return launch_rank<1, true>(x, out, g, st);
        default: return launch_rank<1, false>(x, out, g, st);
    }
}

}  // namespace fz
