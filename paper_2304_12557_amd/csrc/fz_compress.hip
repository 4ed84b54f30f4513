// fz_compress.hip -- per-field compression kernels of libfzmi (gfx950).
//
// k_compress: persistent workgroups of 4 waves take the chunks of one field by
// ticket; each chunk's layers, flags and staged payload come from the device
// code in fz_compress_dev.hpp.  The next chunk's first loads are issued
// before the current chunk is placed.  The device-wide prefix sum of the
// encoder (Sec. 3.4) is a look-back over published chunk sizes: a chunk is
// staged in its workgroup's slot and placed one chunk later, when the sizes
// of the chunks before it are almost always published, so the look-back
// rarely waits; then the slot, still in the cache, is copied to the chunk's
// offset.  The grid's last workgroup to finish settles the status word.  REL
// mode runs k_minmax first (the value range, plus k_init's work), and
// k_compress folds the range into the eb parameters itself.
#include <hip/hip_runtime.h>

#include "fz.h"
#include "fz_compress_dev.hpp"
#include "fz_kernels.hpp"

namespace fz {

// rel_eb > 0: a REL compression whose range pass (k_minmax) left nparts
// partial ranges; every workgroup folds them itself into the eb parameters
// (the same bits everywhere) and workgroup 0 writes them to the header, so
// no separate launch sits between the range pass and this kernel.
template <int RANK, bool VEC4, int QM>
__global__ __launch_bounds__(256, 2) void k_compress(const float* __restrict__ x, uint8_t* __restrict__ out,
                                                     uint8_t* __restrict__ scratch, Geom g, double rel_eb, int nparts)
{
    __shared__ CompressLds S;
    Scratch* scr = reinterpret_cast<Scratch*>(scratch);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: keep it scalar
    Quant inv;
    if (rel_eb > 0.0) {
        const RelParams r = fold_params(scratch, g, rel_eb, nparts);
        if (blockIdx.x == 0 && threadIdx.x == 0) write_params(out, scratch, g, r);
        if (r.status) return;  // the same in every workgroup
        inv = Quant{r.inv, 0u, 0u};
    } else {
        if (scr->pre_status) return;  // set before this launch: uniform across the grid
        inv = quant_of(out);
    }
    uint8_t* slot = scratch + g.scr_stage + kStageSlotBytes * (int64_t)blockIdx.x;

    if (threadIdx.x == 0) {
        S.ticket = atomicAdd(&scr->ticket, 1u);
        S.err = 0;
        S.arrived = 0;
    }
    __syncthreads();
    int64_t c = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)S.ticket);
    if (c >= g.n_chunks) {  // the others took every chunk
        finish_if_last(out, scratch);
        return;
    }
    float h[32], v[32];
    Lane l = lane_geo<RANK>(g, c, lane);
    prefetch<RANK, VEC4>(x, g, l, wave, h, v, swept_down<RANK>(wave));
    int64_t pend = -1;  // the chunk staged in this workgroup's slot, not yet placed
    uint32_t pend_units = 0;

    for (;;) {
        // the next chunk's ticket, taken now so that its return has the whole
        // layer to arrive
        uint32_t tk;  // thread 0 only: a value on the other lanes would need a copy that waits for the atomic
        if (threadIdx.x == 0) tk = atomicAdd(&scr->ticket, 1u);
        uint64_t F[16], myflag;
        // wave priority: the layer at the lowest, the serial part after it
        // (look-back, barrier, placement, staging) at a higher one, so that
        // its few instructions issue first when the CU's other workgroup is in
        // its layer (measured: 512^3 compression about 2 us faster)
        __builtin_amdgcn_s_setprio(0);
        const int nout = chunk_layer<RANK, VEC4, QM>(x, scratch, g, c, l, wave, lane, inv, h, v, S, F, myflag);
        __builtin_amdgcn_s_setprio(3);
        // the previous chunk's offset: wave 0 looks back while the other waves finish their layers
        if (pend >= 0 && wave == 0) place_lookback(out, scratch, g, pend, pend_units, S, lane);
        if (threadIdx.x == 0) S.ticket = tk;
        __syncthreads();
        const int64_t cn = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)S.ticket);
        if (cn < g.n_chunks) {  // start loading the next chunk while this one is placed
            l = lane_geo<RANK>(g, cn, lane);
            prefetch<RANK, VEC4>(x, g, l, wave, h, v, swept_down<RANK>(wave));
        } else {  // defined on every path: otherwise the values of this chunk's
                  // last step stay live across the placement and are spilled
#pragma unroll
            for (int i = 0; i < 32; i++) { h[i] = 0.0f; v[i] = 0.0f; }
        }
        const uint32_t units = chunk_units(S);  // published by the chunk's last layer
        if (pend >= 0) place_copy(out, g, pend_units, slot, S);
        stage_chunk<RANK, VEC4, QM>(x, out, scratch, g, c, wave, lane, inv, F, myflag, nout, S, slot);
        pend = c;
        pend_units = units;
        if (cn >= g.n_chunks) break;
        c = cn;
        __syncthreads();  // the LDS counts and bricks are reused by the next chunk
    }
    if (wave == 0) place_lookback(out, scratch, g, pend, pend_units, S, lane);
    __syncthreads();  // the staged payload and its offset are complete
    place_copy(out, g, pend_units, slot, S);
    finish_if_last(out, scratch);
}

__global__ __launch_bounds__(256) void k_init(uint8_t* __restrict__ out, uint8_t* __restrict__ scratch, Geom g,
                                              HeaderImage h)
{
    init_field(out, scratch, g, h, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// the range pass; with `init` it also does k_init's work (a REL compression
// starts with it)
__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ x, int64_t n, uint8_t* __restrict__ out,
                                                uint8_t* __restrict__ scratch, Geom g, HeaderImage h, int init)
{
    if (init)
        init_field(out, scratch, g, h, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
    minmax_block(x, n, scratch, g, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_params(uint8_t* __restrict__ out, uint8_t* __restrict__ scratch, Geom g,
                                                double eb, int nparts)
{
    params_field(out, scratch, g, eb, nparts);
}

// ----------------------------------------------------------------- launch
int64_t minmax_blocks(int64_t n)
{
    int64_t blocks = (n / 4 + 255) / 256;
    if (blocks > kMinmaxBlocks) blocks = kMinmaxBlocks;
    return blocks < 1 ? 1 : blocks;
}

static hipError_t mark(hipEvent_t e, hipStream_t st) { return e ? hipEventRecord(e, st) : hipSuccess; }

// Whether the compression kernels may read the field with 16-byte loads (the
// VEC4 instantiations): whenever its values are 4-byte aligned, whatever the
// row length.  gfx950 buffer loads need only 4-byte alignment, and their range
// is checked per dword (measured: a 16-byte load straddling the end of the
// range returns the dwords inside it and zeros for the rest), so a load that
// runs past the field's last value still returns that value.  The values a
// lane reads past its chunk's rows belong to other chunks and are masked.
bool vec_loads(const void* x) { return (reinterpret_cast<uintptr_t>(x) & 3) == 0; }

template <int RANK, bool VEC4, int QM>
static hipError_t launch_rank(const float* x, uint8_t* out, uint8_t* scr, const Geom& g, hipStream_t st,
                              const Timing* t = nullptr, double rel_eb = 0.0, int nparts = 0)
{
    // persistent grid: as many workgroups as stay resident, at most one per chunk
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_compress<RANK, VEC4, QM>, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t grid = (int64_t)cus * per_cu;  // one staging slot per workgroup: at most kStageSlots
    if (grid > kStageSlots) grid = kStageSlots;
    if (grid > g.n_chunks) grid = g.n_chunks;
    hipError_t e;
    if (t && (e = mark(t->main_begin, st)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_compress<RANK, VEC4, QM>), dim3((unsigned)grid), dim3(256), 0, st, x, out, scr, g, rel_eb,
                       nparts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (t && (e = mark(t->main_end, st)) != hipSuccess) return e;
    return t ? mark(t->done, st) : hipSuccess;
}

static hipError_t launch_init(uint8_t* out, uint8_t* scr, const Geom& g, const HeaderImage& h, hipStream_t st)
{
    const int64_t init_threads = g.n_chunks > kHeaderBytes / 4 ? g.n_chunks : kHeaderBytes / 4;
    const unsigned init_blocks = (unsigned)((init_threads + 255) / 256 < 1024 ? (init_threads + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_init, dim3(init_blocks), dim3(256), 0, st, out, scr, g, h);
    return hipGetLastError();
}

// the compression kernel on the integer buffer at g.q_off (scratch inside the output buffer)
static hipError_t launch_main_int(uint8_t* out, const Geom& g, hipStream_t st)
{
    // the integer buffer is 256-byte aligned: 16-byte loads (they need only
    // 4-byte alignment, see vec_loads)
    const float* qf = reinterpret_cast<const float*>(out + g.q_off);
    uint8_t* scr = out + g.scratch_off;
    switch (g.rank) {
        case 3: return launch_rank<3, true, kQuantInt>(qf, out, scr, g, st);
        case 2: return launch_rank<2, true, kQuantInt>(qf, out, scr, g, st);
        default: return launch_rank<1, true, kQuantInt>(qf, out, scr, g, st);
    }
}

hipError_t launch_compress_f64(const double* x, uint8_t* out, const Geom& g, const HeaderImage& h, int mode,
                               double eb, hipStream_t st)
{
    hipError_t e = launch_init(out, out + g.scratch_off, g, h, st);
    if (e != hipSuccess) return e;
    if ((e = launch_f64_front(x, out, g, mode, eb, st)) != hipSuccess) return e;
    return launch_main_int(out, g, st);
}

// the value range and the eb parameters of the relative bound (after k_init)
static hipError_t launch_range(const float* x, uint8_t* out, uint8_t* scr, const Geom& g, double eb, hipStream_t st)
{
    const int64_t n = g.n[0] * g.n[1] * g.n[2];
    const int64_t blocks = minmax_blocks(n);
    hipLaunchKernelGGL(k_minmax, dim3((unsigned)blocks), dim3(256), 0, st, x, n, out, scr, g, HeaderImage{}, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_params, dim3(1), dim3(256), 0, st, out, scr, g, eb, (int)blocks);
    return hipGetLastError();
}

hipError_t launch_compress_global(const float* x, uint8_t* out, const Geom& g, const HeaderImage& h, int mode,
                                  double eb, hipStream_t st)
{
    uint8_t* scr = out + g.scratch_off;
    hipError_t e = launch_init(out, scr, g, h, st);
    if (e != hipSuccess) return e;
    if (mode == FZ_EB_REL && (e = launch_range(x, out, scr, g, eb, st)) != hipSuccess) return e;
    if ((e = launch_face(x, out, g, st)) != hipSuccess) return e;
    return launch_main_int(out, g, st);
}

hipError_t launch_compress(const float* x, uint8_t* out, uint8_t* scr, const Geom& g, const HeaderImage& h, int mode,
                           double eb, hipStream_t st, const Timing* t)
{
    // REL: the range pass also initializes (the header image, the scratch), and
    // the compression kernel folds the range itself: 2 launches
    hipError_t e;
    double rel_eb = 0.0;
    int nparts = 0;
    if (mode == FZ_EB_REL) {
        if (t && (e = mark(t->range_begin, st)) != hipSuccess) return e;
        const int64_t n = g.n[0] * g.n[1] * g.n[2];
        const int64_t blocks = minmax_blocks(n);
        hipLaunchKernelGGL(k_minmax, dim3((unsigned)blocks), dim3(256), 0, st, x, n, out, scr, g, h, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        rel_eb = eb;
        nparts = (int)blocks;
    } else {
        if ((e = launch_init(out, scr, g, h, st)) != hipSuccess) return e;
        if (t && (e = mark(t->range_begin, st)) != hipSuccess) return e;
    }
    const bool vec4 = vec_loads(x);
    if (mode == FZ_EB_PWREL) {
        switch (g.rank * 2 + (vec4 ? 1 : 0)) {
            case 7: return launch_rank<3, true, kQuantPw>(x, out, scr, g, st, t);
            case 6: return launch_rank<3, false, kQuantPw>(x, out, scr, g, st, t);
            case 5: return launch_rank<2, true, kQuantPw>(x, out, scr, g, st, t);
            case 4: return launch_rank<2, false, kQuantPw>(x, out, scr, g, st, t);
            case 3: return launch_rank<1, true, kQuantPw>(x, out, scr, g, st, t);
            default: return launch_rank<1, false, kQuantPw>(x, out, scr, g, st, t);
        }
    }
    switch (g.rank * 2 + (vec4 ? 1 : 0)) {
        case 7: return launch_rank<3, true, kQuantGrid>(x, out, scr, g, st, t, rel_eb, nparts);
        case 6: return launch_rank<3, false, kQuantGrid>(x, out, scr, g, st, t, rel_eb, nparts);
        case 5: return launch_rank<2, true, kQuantGrid>(x, out, scr, g, st, t, rel_eb, nparts);
        case 4: return launch_rank<2, false, kQuantGrid>(x, out, scr, g, st, t, rel_eb, nparts);
        case 3: return launch_rank<1, true, kQuantGrid>(x, out, scr, g, st, t, rel_eb, nparts);
        default: return launch_rank<1, false, kQuantGrid>(x, out, scr, g, st, t, rel_eb, nparts);
    }
}

}  // namespace fz
