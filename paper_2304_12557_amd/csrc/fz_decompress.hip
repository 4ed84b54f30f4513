// fz_decompress.hip -- per-field decompression kernels of libfzmi (gfx950):
// one wave per chunk, or for fields with few chunks a workgroup of 4 waves
// per chunk (one per layer), running the device code of fz_decompress_dev.hpp.
#include <hip/hip_runtime.h>

#include "fz_decompress_dev.hpp"
#include "fz_kernels.hpp"

namespace fz {

template <int RANK, bool VEC4>
__global__ __launch_bounds__(64, 2) void k_decompress(const uint8_t* __restrict__ s, uint64_t sb,
                                                      float* __restrict__ y, Geom g, uint32_t* d_err)
{
    __shared__ float tile[kTileFloats];
    decompress_chunk_any<RANK, VEC4>(s, sb, y, g, d_err, blockIdx.x, threadIdx.x, tile);
}

// the same with a workgroup of NW waves per chunk, each on 4/NW layers
// (fields with few chunks; launched with NW = 4).  Both forms are held to 2
// waves per SIMD: left to itself the compiler took 258 registers for the 3-D
// form, which allows only 1 (512^3 decompression 152 -> 132 us at 2).
template <int RANK, bool VEC4, int NW>
__global__ __launch_bounds__(64 * NW, 2) void k_decompress_split(const uint8_t* __restrict__ s, uint64_t sb,
                                                              float* __restrict__ y, Geom g, uint32_t* d_err)
{
    __shared__ float tiles[NW][kTileFloats];
    __shared__ int xch[NW * 2048];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    decompress_chunk_any<RANK, VEC4, NW>(s, sb, y, g, d_err, blockIdx.x, threadIdx.x & 63, tiles[wave], wave, xch);
}

__global__ void k_set_u32(uint32_t* p, uint32_t v)
{
    if (threadIdx.x == 0) *p = v;
}

// fields of at most this many chunks are decompressed with 4 waves per chunk
constexpr int64_t kSplitChunks = 512;

template <int RANK, bool VEC4>
static hipError_t launch_rank(const uint8_t* s, uint64_t sb, float* y, const Geom& g, uint32_t* d_err, hipStream_t st)
{
    // Up to 512 chunks (2048 waves, what the chip holds at 2 per SIMD) a chunk
    // gets 4 waves: its latency, not the VALU throughput, then sets the time.
    // Beyond, the single wave per chunk is faster (measured: a 2-wave form
    // lost everywhere, since 2 waves on one SIMD share its VALU and the split
    // adds a decode pass).
    if (g.n_chunks <= kSplitChunks)
        hipLaunchKernelGGL((k_decompress_split<RANK, VEC4, kLayers>), dim3((unsigned)g.n_chunks), dim3(64 * kLayers), 0,
                           st, s, sb, y, g, d_err);
    else
        hipLaunchKernelGGL((k_decompress<RANK, VEC4>), dim3((unsigned)g.n_chunks), dim3(64), 0, st, s, sb, y, g, d_err);
    return hipGetLastError();
}

hipError_t launch_decompress(const uint8_t* s, uint64_t sb, float* y, const Geom& g, uint32_t* d_err, hipStream_t st)
{
    if (d_err) {
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, st, d_err, 0u);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const bool vec4 = (reinterpret_cast<uintptr_t>(y) & 15) == 0 && (g.rank == 1 || (g.n[g.rank - 1] & 3) == 0);
    switch (g.rank * 2 + (vec4 ? 1 : 0)) {
        case 7: return launch_rank<3, true>(s, sb, y, g, d_err, st);
        case 6: return launch_rank<3, false>(s, sb, y, g, d_err, st);
        case 5: return launch_rank<2, true>(s, sb, y, g, d_err, st);
        case 4: return launch_rank<2, false>(s, sb, y, g, d_err, st);
        case 3: return launch_rank<1, true>(s, sb, y, g, d_err, st);
        default: return launch_rank<1, false>(s, sb, y, g, d_err, st);
    }
}

}  // namespace fz
