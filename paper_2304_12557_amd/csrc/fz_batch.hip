// fz_batch.hip -- batched compression and decompression of many fields of
// uneven rank and size (libfzmi's batch layer).
//
// A plan holds, in device memory, one descriptor per field and a chunk -> field
// table over the concatenated chunks of all fields.  Running a compression
// plan enqueues a fixed sequence of launches whatever the number of fields:
//   init (all fields) -> value range + eb (REL fields) -> one persistent
//   compression launch per (rank, row-alignment) class present (at most six,
//   usually three), each over every chunk of every field of its class, which
//   also places the chunks -> the final status word of each field
// and a decompression plan one launch over every chunk of every field.  Each
// field's bytes are exactly those of the per-field call: the per-chunk and
// per-field device code is the same (fz_compress_dev.hpp,
// fz_decompress_dev.hpp), only the mapping of workgroups to fields differs.
// Nothing is allocated, copied from the host or synchronized while a plan
// runs, so a run can be captured in a hipGraph and replayed.
//
// The launch shapes (persistent workgroups per CU, range-pass blocks per
// field) come from a small autotuner that times
// the candidates on the plan's own fields; the chunk shapes are part of the
// stream format and stay fixed, so tuning never changes a byte.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fz.h"
#include "fz_compress_dev.hpp"
#include "fz_batch.hpp"
#include "fz_decompress_dev.hpp"
#include "fz_kernels.hpp"

namespace fz {

// ---------------------------------------------------------------- kernels
__global__ __launch_bounds__(256) void k_batch_init(const CompressJob* __restrict__ jobs, int n_jobs,
                                                    uint32_t* __restrict__ ticket)
{
    if ((int)blockIdx.x == n_jobs) {
        if (threadIdx.x < 8) ticket[threadIdx.x] = 0u;  // one ticket counter per class
        return;
    }
    const CompressJob& J = jobs[blockIdx.x];
    init_field(J.out, J.out + J.g.scratch_off, J.g, J.h, threadIdx.x, 256);
}

__global__ __launch_bounds__(256) void k_batch_minmax(const CompressJob* __restrict__ jobs,
                                                      const int32_t* __restrict__ mm_job)
{
    const int j = mm_job[blockIdx.x];
    const CompressJob& J = jobs[j];
    minmax_block(J.x, J.g.n[0] * J.g.n[1] * J.g.n[2], J.out + J.g.scratch_off, J.g, (int64_t)blockIdx.x - J.mm0,
                 J.mm_blocks);
}

__global__ __launch_bounds__(256) void k_batch_params(const CompressJob* __restrict__ jobs)
{
    const CompressJob& J = jobs[blockIdx.x];
    if (J.rel) params_field(J.out, J.out + J.g.scratch_off, J.g, J.eb, (int)J.mm_blocks);
}

// One persistent launch per (rank, alignment) class over the chunks of every
// field of that class: tickets run over the class's part of the chunk table,
// which maps a ticket to its field.  Within a field the next chunk's first
// loads are issued before the current one is placed, as in the per-field
// kernel, and chunks are placed as there: staged in the workgroup's slot of
// the plan's staging area and copied to their offset one chunk later, after
// a look-back over the field's published chunk sizes.  Fields whose REL pass
// failed are skipped.  (One instantiation per launch keeps the register
// budget of the per-field kernel; a kernel holding all six would spill.)
template <int RANK, bool VEC4>
__global__ __launch_bounds__(256, 2) void k_batch_compress(const CompressJob* __restrict__ jobs,
                                                           const int32_t* __restrict__ chunk_job, int64_t total,
                                                           uint32_t* __restrict__ ticket, uint8_t* __restrict__ stage)
{
    __shared__ CompressLds S;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint8_t* slot = stage + kStageSlotBytes * (int64_t)blockIdx.x;
    if (threadIdx.x == 0) {
        S.ticket = atomicAdd(ticket, 1u);
        S.err = 0;
        S.arrived = 0;
    }
    __syncthreads();
    int64_t t = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)S.ticket);
    if (t >= total) return;
    int j = __builtin_amdgcn_readfirstlane(chunk_job[t]);
    float h[32], v[32];
    bool loaded = false;
    int pend_j = -1;  // field and chunk staged in this workgroup's slot, not yet placed
    int64_t pend_c = 0;
    uint32_t pend_units = 0;
    for (;;) {
        const CompressJob& J = jobs[j];
        const Geom g = J.g;
        const int64_t c = t - J.chunk0;
        uint8_t* scr = J.out + g.scratch_off;
        const bool skip = reinterpret_cast<const Scratch*>(scr)->pre_status != 0;
        const Quant inv = quant_of(J.out);
        const Lane l = lane_geo<RANK>(g, c, lane);
        if (!skip && !loaded) prefetch<RANK, VEC4>(J.x, g, l, wave, h, v, swept_down<RANK>(wave));
        uint32_t tk;  // the next ticket, taken early by thread 0 (its return has the layer to arrive)
        if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
        uint64_t F[16], myflag = 0;
        int nout = 0;
        if (!skip) nout = chunk_layer<RANK, VEC4>(J.x, scr, g, c, l, wave, lane, inv, h, v, S, F, myflag);
        if (pend_j >= 0 && wave == 0) {  // the previous chunk's offset, while the other waves finish their layers
            const CompressJob& P = jobs[pend_j];
            place_lookback(P.out, P.out + P.g.scratch_off, P.g, pend_c, pend_units, S, lane);
        }
        if (threadIdx.x == 0) S.ticket = tk;
        __syncthreads();
        const int64_t tn = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)S.ticket);
        const int jn = tn < total ? __builtin_amdgcn_readfirstlane(chunk_job[tn]) : -1;
        loaded = false;
        if (jn == j && !skip) {  // same field: start the next chunk's loads now
            const Lane ln = lane_geo<RANK>(g, tn - J.chunk0, lane);
            prefetch<RANK, VEC4>(J.x, g, ln, wave, h, v, swept_down<RANK>(wave));
            loaded = true;
        }
        if (!loaded) {  // defined on every path, so that no value of this chunk stays live into the next
#pragma unroll
            for (int i = 0; i < 32; i++) { h[i] = 0.0f; v[i] = 0.0f; }
        }
        const uint32_t units = skip ? 0u : chunk_units(S);  // published by the chunk's last layer
        if (pend_j >= 0) place_copy(jobs[pend_j].out, jobs[pend_j].g, pend_units, slot, S);
        pend_j = -1;
        if (!skip) {
            stage_chunk<RANK, VEC4>(J.x, J.out, scr, g, c, wave, lane, inv, F, myflag, nout, S, slot);
            pend_j = j;
            pend_c = c;
            pend_units = units;
        }
        if (tn >= total) break;
        t = tn;
        j = jn;
        __syncthreads();
    }
    if (pend_j >= 0) {
        const CompressJob& P = jobs[pend_j];
        if (wave == 0) place_lookback(P.out, P.out + P.g.scratch_off, P.g, pend_c, pend_units, S, lane);
        __syncthreads();  // the staged payload and its offset are complete
        place_copy(P.out, P.g, pend_units, slot, S);
    }
}

// after every chunk of every field is placed: each field's final status word
__global__ __launch_bounds__(64) void k_batch_finish(const CompressJob* __restrict__ jobs)
{
    const CompressJob& J = jobs[blockIdx.x];
    if (threadIdx.x == 0) finish_field(J.out, J.out + J.g.scratch_off);
}

__global__ __launch_bounds__(256) void k_batch_clear_err(const DecompressJob* __restrict__ jobs, int n_jobs)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_jobs && jobs[j].err) *jobs[j].err = 0u;
}

__global__ __launch_bounds__(64, 2) void k_batch_decompress(const DecompressJob* __restrict__ jobs,
                                                         const int32_t* __restrict__ chunk_job)
{
    __shared__ float tile[kTileFloats];
    const DecompressJob& J = jobs[chunk_job[blockIdx.x]];
    const int64_t c = (int64_t)blockIdx.x - J.chunk0;
    const int lane = threadIdx.x;
    switch (J.key) {
        case 7: decompress_chunk_any<3, true>(J.s, J.s_bytes, J.y, J.g, J.err, c, lane, tile); break;
        case 6: decompress_chunk_any<3, false>(J.s, J.s_bytes, J.y, J.g, J.err, c, lane, tile); break;
        case 5: decompress_chunk_any<2, true>(J.s, J.s_bytes, J.y, J.g, J.err, c, lane, tile); break;
        case 4: decompress_chunk_any<2, false>(J.s, J.s_bytes, J.y, J.g, J.err, c, lane, tile); break;
        case 3: decompress_chunk_any<1, true>(J.s, J.s_bytes, J.y, J.g, J.err, c, lane, tile); break;
        default: decompress_chunk_any<1, false>(J.s, J.s_bytes, J.y, J.g, J.err, c, lane, tile); break;
    }
}

// ------------------------------------------------------------------- plans
namespace {

// launch class of a field: rank and whether whole 16-byte accesses apply
// (decompression: 16-byte aligned output rows of whole 16-byte pieces;
// compression: 4-byte aligned input, vec_loads)
int vec_key(const void* p, const Geom& g)
{
    const bool vec4 = (reinterpret_cast<uintptr_t>(p) & 15) == 0 && (g.rank == 1 || (g.n[g.rank - 1] & 3) == 0);
    return g.rank * 2 + (vec4 ? 1 : 0);
}

int compress_key(const void* p, const Geom& g) { return g.rank * 2 + (vec_loads(p) ? 1 : 0); }


}  // namespace

int cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 1;
    return cus;
}

// Host image of a plan's device tables for its current tuning: ticket
// counters, job table, chunk -> job, range-pass block -> job.  `cap_mm` is
// the number of block entries reserved (at least the current count).
size_t plan_layout(Plan* P, int64_t cap_mm, std::vector<uint8_t>* img)
{
    std::vector<int32_t> chunk_job(P->total_chunks), mm_job;
    int64_t mm = 0;
    for (int j = 0; j < P->n_jobs; j++) {
        if (P->compress) {
            CompressJob& J = P->cjobs[j];
            for (int64_t c = 0; c < J.g.n_chunks; c++) chunk_job[J.chunkg + c] = j;
            J.mm0 = mm;
            J.mm_blocks = 0;
            if (J.rel) {
                int64_t b = minmax_blocks(J.g.n[0] * J.g.n[1] * J.g.n[2]);
                if (b > P->tune.mm_cap) b = P->tune.mm_cap;
                J.mm_blocks = b;
                for (int64_t i = 0; i < b; i++) mm_job.push_back(j);
                mm += b;
            }
        } else {
            const DecompressJob& J = P->djobs[j];
            for (int64_t c = 0; c < J.g.n_chunks; c++) chunk_job[J.chunk0 + c] = j;
        }
    }
    P->total_mm = mm;
    if (cap_mm < mm) cap_mm = mm;
    const size_t job_bytes = P->compress ? sizeof(CompressJob) * P->n_jobs : sizeof(DecompressJob) * P->n_jobs;
    P->off_jobs = 256;
    P->off_chunk = (P->off_jobs + job_bytes + 255) / 256 * 256;
    P->off_mm = (P->off_chunk + 4 * (size_t)P->total_chunks + 255) / 256 * 256;
    const size_t bytes = P->off_mm + 4 * (size_t)(cap_mm > 0 ? cap_mm : 1);
    if (img) {
        img->assign(bytes, 0);
        const void* src =
            P->compress ? static_cast<const void*>(P->cjobs.data()) : static_cast<const void*>(P->djobs.data());
        std::memcpy(img->data() + P->off_jobs, src, job_bytes);
        std::memcpy(img->data() + P->off_chunk, chunk_job.data(), 4 * chunk_job.size());
        if (mm > 0) std::memcpy(img->data() + P->off_mm, mm_job.data(), 4 * mm_job.size());
    }
    return bytes;
}

// Point the plan at a device area that holds (or will hold) its image.
void plan_bind(Plan* P, void* dev)
{
    uint8_t* base = static_cast<uint8_t*>(dev);
    P->d_ticket = reinterpret_cast<uint32_t*>(base);
    P->d_jobs = base + P->off_jobs;
    P->d_chunk_job = reinterpret_cast<int32_t*>(base + P->off_chunk);
    P->d_mm_job = reinterpret_cast<int32_t*>(base + P->off_mm);
}

// (Re)build the device tables of a standalone plan for its current tuning:
// one device block, sized for the largest tuning (its addresses never change,
// so launches captured in a graph stay valid until the plan is destroyed;
// tune before capturing, since a capture bakes the tuning in).
int upload(Plan* P)
{
    std::vector<uint8_t> img;
    const size_t bytes = plan_layout(P, P->mm_max, &img);
    if (!P->dev && hipMalloc(&P->dev, bytes) != hipSuccess) {
        P->dev = nullptr;
        return FZ_ERR_HIP;
    }
    plan_bind(P, P->dev);
    return hipMemcpy(P->dev, img.data(), bytes, hipMemcpyHostToDevice) == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

hipError_t plan_run(const Plan* P, hipStream_t st)
{
    hipError_t e;
    if (!P->compress) {
        const DecompressJob* jobs = static_cast<const DecompressJob*>(P->d_jobs);
        hipLaunchKernelGGL(k_batch_clear_err, dim3((P->n_jobs + 255) / 256), dim3(256), 0, st, jobs, P->n_jobs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_batch_decompress, dim3((unsigned)P->total_chunks), dim3(64), 0, st, jobs, P->d_chunk_job);
        return hipGetLastError();
    }
    const CompressJob* jobs = static_cast<const CompressJob*>(P->d_jobs);
    hipLaunchKernelGGL(k_batch_init, dim3(P->n_jobs + 1), dim3(256), 0, st, jobs, P->n_jobs, P->d_ticket);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (P->any_rel) {
        hipLaunchKernelGGL(k_batch_minmax, dim3((unsigned)P->total_mm), dim3(256), 0, st, jobs, P->d_mm_job);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_batch_params, dim3(P->n_jobs), dim3(256), 0, st, jobs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int key = 2; key < 8; key++) {
        const int64_t n = P->class_chunks[key];
        if (n == 0) continue;
        int64_t grid = (int64_t)P->cus * P->tune.per_cu;
        if (grid > stage_slots(P->cus)) grid = stage_slots(P->cus);
        if (grid > n) grid = n;
        const int32_t* tab = P->d_chunk_job + P->class_off[key];
        uint32_t* tk = P->d_ticket + key;
        uint8_t* sg = static_cast<uint8_t*>(P->d_stage);
        switch (key) {
            case 7: hipLaunchKernelGGL((k_batch_compress<3, true>), dim3((unsigned)grid), dim3(256), 0, st, jobs, tab, n, tk, sg); break;
            case 6: hipLaunchKernelGGL((k_batch_compress<3, false>), dim3((unsigned)grid), dim3(256), 0, st, jobs, tab, n, tk, sg); break;
            case 5: hipLaunchKernelGGL((k_batch_compress<2, true>), dim3((unsigned)grid), dim3(256), 0, st, jobs, tab, n, tk, sg); break;
            case 4: hipLaunchKernelGGL((k_batch_compress<2, false>), dim3((unsigned)grid), dim3(256), 0, st, jobs, tab, n, tk, sg); break;
            case 3: hipLaunchKernelGGL((k_batch_compress<1, true>), dim3((unsigned)grid), dim3(256), 0, st, jobs, tab, n, tk, sg); break;
            default: hipLaunchKernelGGL((k_batch_compress<1, false>), dim3((unsigned)grid), dim3(256), 0, st, jobs, tab, n, tk, sg); break;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_finish, dim3(P->n_jobs), dim3(64), 0, st, jobs);
    return hipGetLastError();
}

int plan_compress(Plan* Pp, int n, const fz_compress_job* jobs)
{
    Plan& P = *Pp;
    if (n < 1 || !jobs) return FZ_ERR_ARG;
    P.compress = true;
    P.n_jobs = n;
    for (int k = 0; k < 8; k++) P.class_off[k] = P.class_chunks[k] = 0;
    P.dev = nullptr;
    P.d_stage = nullptr;
    P.cus = cu_count();
    P.tune = Tuning{2, kMinmaxBlocks};
    P.any_rel = false;
    P.mm_max = 0;
    P.cjobs.clear();
    P.djobs.clear();
    int64_t chunks = 0;
    for (int i = 0; i < n; i++) {
        const fz_compress_job& q = jobs[i];
        CompressJob J;
        std::memset(&J, 0, sizeof(J));
        const double eb = q.eb;
        if (!q.d_in || !q.d_out || !make_geom((int)q.dims.rank, q.dims.n, &J.g)) return FZ_ERR_ARG;
        if (!aligned_to(q.d_in, 4) || !aligned_to(q.d_out, 256)) return FZ_ERR_ARG;
        if (!(eb > 0.0) || !std::isfinite(eb) || (q.eb_mode != FZ_EB_ABS && q.eb_mode != FZ_EB_REL)) return FZ_ERR_ARG;
        float ebx2 = 0.0f, inv = 0.0f;
        if (q.eb_mode == FZ_EB_ABS && !abs_params(eb, &ebx2, &inv)) return FZ_ERR_EB_RANGE;
        J.x = q.d_in;
        J.out = static_cast<uint8_t*>(q.d_out);
        J.h = header_image(J.g, eb, q.eb_mode, ebx2, inv);
        J.eb = eb;
        J.rel = q.eb_mode == FZ_EB_REL;
        J.key = compress_key(q.d_in, J.g);
        J.chunk0 = P.class_chunks[J.key];
        P.class_chunks[J.key] += J.g.n_chunks;
        chunks += J.g.n_chunks;
        P.any_rel |= J.rel != 0;
        if (J.rel) P.mm_max += minmax_blocks(J.g.n[0] * J.g.n[1] * J.g.n[2]);
        P.cjobs.push_back(J);
    }
    if (chunks >= (1ll << 31)) return FZ_ERR_ARG;
    P.total_chunks = chunks;
    int64_t off = 0;
    for (int key = 0; key < 8; key++) {  // the chunk table is ordered by class
        P.class_off[key] = off;
        off += P.class_chunks[key];
    }
    for (CompressJob& J : P.cjobs) J.chunkg = P.class_off[J.key] + J.chunk0;
    return FZ_OK;
}

int plan_decompress(Plan* Pp, int n, const fz_decompress_job* jobs)
{
    Plan& P = *Pp;
    if (n < 1 || !jobs) return FZ_ERR_ARG;
    P.compress = false;
    P.n_jobs = n;
    for (int k = 0; k < 8; k++) P.class_off[k] = P.class_chunks[k] = 0;
    P.dev = nullptr;
    P.d_stage = nullptr;
    P.cus = cu_count();
    P.tune = Tuning{2, kMinmaxBlocks};
    P.any_rel = false;
    P.mm_max = 0;
    P.cjobs.clear();
    P.djobs.clear();
    int64_t chunks = 0;
    for (int i = 0; i < n; i++) {
        const fz_decompress_job& q = jobs[i];
        DecompressJob J;
        std::memset(&J, 0, sizeof(J));
        if (!q.d_stream || !q.d_out || !make_geom((int)q.dims.rank, q.dims.n, &J.g)) return FZ_ERR_ARG;
        if (!aligned_to(q.d_stream, 256) || !aligned_to(q.d_out, 4) || !aligned_to(q.d_err, 4) ||
            q.stream_bytes < (uint64_t)J.g.payload_off)
            return FZ_ERR_ARG;
        J.s = static_cast<const uint8_t*>(q.d_stream);
        J.s_bytes = q.stream_bytes;
        J.y = q.d_out;
        J.err = q.d_err;
        J.key = vec_key(q.d_out, J.g);
        J.chunk0 = chunks;
        chunks += J.g.n_chunks;
        P.djobs.push_back(J);
    }
    if (chunks >= (1ll << 31)) return FZ_ERR_ARG;
    P.total_chunks = chunks;
    return FZ_OK;
}

}  // namespace fz

using namespace fz;

struct fz_batch {
    Plan p;
};

namespace {

int create(fz_batch** out, bool compress, int n, const void* jobs)
{
    if (!out) return FZ_ERR_ARG;
    *out = nullptr;
    fz_batch* b = new (std::nothrow) fz_batch();
    if (!b) return FZ_ERR_ARG;
    int rc = compress ? plan_compress(&b->p, n, static_cast<const fz_compress_job*>(jobs))
                      : plan_decompress(&b->p, n, static_cast<const fz_decompress_job*>(jobs));
    if (rc == FZ_OK) rc = upload(&b->p);
    if (rc == FZ_OK && b->p.compress && hipMalloc(&b->p.d_stage, stage_bytes(b->p.cus)) != hipSuccess) {
        b->p.d_stage = nullptr;
        rc = FZ_ERR_HIP;
    }
    if (rc != FZ_OK) {
        if (b->p.dev) (void)hipFree(b->p.dev);
        delete b;
        return rc;
    }
    *out = b;
    return FZ_OK;
}

}  // namespace

extern "C" {

int fz_batch_create_compress(int n, const fz_compress_job* jobs, fz_batch** out)
{
    return create(out, true, n, jobs);
}

int fz_batch_create_decompress(int n, const fz_decompress_job* jobs, fz_batch** out)
{
    return create(out, false, n, jobs);
}

int fz_batch_run(fz_batch* b, void* stream)
{
    if (!b) return FZ_ERR_ARG;
    return plan_run(&b->p, static_cast<hipStream_t>(stream)) == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_batch_tune(fz_batch* b, void* stream)
{
    if (!b) return FZ_ERR_ARG;
    Plan& P = b->p;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!P.compress) return hipStreamSynchronize(st) == hipSuccess ? FZ_OK : FZ_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FZ_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FZ_ERR_HIP;
    }
    const Tuning cands[] = {{2, kMinmaxBlocks}, {1, kMinmaxBlocks}, {2, 512}, {1, 512}};
    Tuning best = P.tune;
    float best_ms = 1e30f;
    int rc = FZ_OK;
    for (const Tuning& t : cands) {
        P.tune = t;
        if ((rc = upload(&P)) != FZ_OK) break;
        if (plan_run(&P, st) != hipSuccess) { rc = FZ_ERR_HIP; break; }  // warm-up
        float ms = 1e30f;
        for (int r = 0; r < 3 && rc == FZ_OK; r++) {
            float m = 0.0f;
            if (hipEventRecord(e0, st) != hipSuccess || plan_run(&P, st) != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&m, e0, e1) != hipSuccess)
                rc = FZ_ERR_HIP;
            ms = m < ms ? m : ms;
        }
        if (rc != FZ_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P.tune = best;
    const int rc2 = upload(&P);
    return rc != FZ_OK ? rc : rc2;
}

int fz_batch_destroy(fz_batch* b)
{
    if (!b) return FZ_ERR_ARG;
    int rc = FZ_OK;
    if (b->p.dev && hipFree(b->p.dev) != hipSuccess) rc = FZ_ERR_HIP;
    if (b->p.d_stage && hipFree(b->p.d_stage) != hipSuccess) rc = FZ_ERR_HIP;
    delete b;
    return rc;
}

}  // extern "C"
