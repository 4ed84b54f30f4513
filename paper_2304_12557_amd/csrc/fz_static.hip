// fz_static.hip -- the compression entry point that allocates nothing
// (fz_compress_noalloc): the same kernels as fz_compress, with the
// compression's scratch (chunk tickets and sizes, the partial value ranges of
// the REL pass, the staging slots) in a file-scope device array instead of the
// tail of the caller's output buffer.
//
// Each device the library runs on holds its own copy of the array for the
// life of the process.  Its device address is taken once per device, at the
// entry point's first call there (with that device current), and kept: in
// host code the array's name is only a host-side stand-in, so kernels get the
// address from hipGetSymbolAddress, never the name.  Calls on one device
// share the array; every call clears what must start at zero (ticket, status,
// chunk states) with a kernel before use, and calls that overlap on one
// device race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fz.h"
#include "fz_format.hpp"
#include "fz_kernels.hpp"

namespace fz {
namespace {

static_assert(FZ_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
__device__ __align__(256) uint8_t scratch[FZ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices];  // device address of `scratch` on each device, once taken

// the array's address on the current device (taken at the first call there)
hipError_t scratch_ptr(uint8_t** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace fz

using namespace fz;

extern "C" {

int fz_compress_noalloc(const float* d_in, const fz_dims* dims, double eb, int eb_mode, void* d_out, size_t out_bytes,
                        void* stream)
{
    Geom g;
    if (!d_in || !d_out || !dims || !make_geom((int)dims->rank, dims->n, &g) || !aligned_to(d_in, 4) ||
        !aligned_to(d_out, 256))
        return FZ_ERR_ARG;
    if (out_bytes < (size_t)g.stream_bound || g.scr_bytes > (int64_t)FZ_NOALLOC_SCRATCH_BYTES) return FZ_ERR_ARG;
    float ebx2 = 0.0f, inv = 0.0f;
    const int rc = bound_params(eb, eb_mode, &ebx2, &inv);
    if (rc != FZ_OK) return rc;
    uint8_t* scr = nullptr;
    if (scratch_ptr(&scr) != hipSuccess) return FZ_ERR_HIP;
    const HeaderImage h = header_image(g, eb, eb_mode, ebx2, inv);
    const hipError_t e = launch_compress(d_in, static_cast<uint8_t*>(d_out), scr, g, h, eb_mode, eb,
                                         static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

}  // extern "C"
