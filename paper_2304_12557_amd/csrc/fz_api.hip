// fz_api.hip -- the C ABI of libfzmi (declared in include/fz.h): argument
// checks, chunk planning, the stream header image, and the launches.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>

#include "fz.h"
#include "fz_format.hpp"
#include "fz_kernels.hpp"

using namespace fz;

namespace {

bool geom_of(const fz_dims* d, Geom* g)
{
    if (!d) return false;
    return make_geom((int)d->rank, d->n, g);
}

void put_bytes(HeaderImage& h, int off, const void* src, int n) { std::memcpy(reinterpret_cast<uint8_t*>(h.w) + off, src, n); }

}  // namespace

namespace fz {

HeaderImage header_image_f64(const Geom& g, double eb, int mode, double ebx2, double inv)
{
    HeaderImage h = header_image(g, eb, mode, (float)ebx2, (float)inv);
    const uint8_t dtype = 1;
    put_bytes(h, kOffDtype, &dtype, 1);
    put_bytes(h, kOffEbx2F64, &ebx2, 8);
    put_bytes(h, kOffInvF64, &inv, 8);
    return h;
}

HeaderImage header_image(const Geom& g, double eb, int mode, float ebx2, float inv)
{
    HeaderImage h;
    std::memset(&h, 0, sizeof(h));
    const uint32_t magic = kMagic;
    const uint16_t ver = kVersion, hb = kHeaderBytes;
    put_bytes(h, kOffMagic, &magic, 4);
    put_bytes(h, kOffVersion, &ver, 2);
    put_bytes(h, kOffHdrBytes, &hb, 2);
    const uint8_t dtype = 0, rank = (uint8_t)g.rank, m = (uint8_t)mode;
    put_bytes(h, kOffDtype, &dtype, 1);
    put_bytes(h, kOffRank, &rank, 1);
    put_bytes(h, kOffEbMode, &m, 1);
    for (int i = 0; i < 3; i++) {
        const uint64_t n = (uint64_t)g.n[i];
        put_bytes(h, kOffDims + 8 * i, &n, 8);
        const uint16_t b = (uint16_t)g.box[i];
        put_bytes(h, kOffChunk + 2 * i, &b, 2);
    }
    put_bytes(h, kOffEbUser, &eb, 8);
    put_bytes(h, kOffEbx2, &ebx2, 4);
    put_bytes(h, kOffInv, &inv, 4);
    const uint32_t nch = (uint32_t)g.n_chunks;
    put_bytes(h, kOffNChunks, &nch, 4);
    return h;
}

// eb parameters of an absolute bound: ebx2 = fp32(2 eb), inv = fp32(1 / (double)ebx2);
// false if they are unusable (2 eb not a normal fp32, or inv not finite)
bool abs_params(double eb, float* ebx2, float* inv)
{
    *ebx2 = (float)(2.0 * eb);
    *inv = (float)(1.0 / (double)*ebx2);
    return *ebx2 >= FLT_MIN && std::isfinite(*ebx2) && std::isfinite(*inv) && *inv > 0.0f;
}

int bound_params(double eb, int mode, float* ebx2, float* inv)
{
    *ebx2 = 0.0f;
    *inv = 0.0f;
    if (!(eb > 0.0) || !std::isfinite(eb)) return FZ_ERR_ARG;
    switch (mode) {
        case FZ_EB_ABS: return abs_params(eb, ebx2, inv) ? FZ_OK : FZ_ERR_EB_RANGE;
        case FZ_EB_REL: return FZ_OK;
        case FZ_EB_PWREL: {
            // the largest step whose half keeps every value within the
            // relative bound, also across a binade boundary (where the
            // mantissa's weight doubles): S / 2^24 <= eb / (1 + eb)
            const double step = std::floor(eb * 16777216.0 / (1.0 + eb));
            if (!(step >= 2.0 && step < 16777216.0)) return FZ_ERR_EB_RANGE;
            *ebx2 = (float)step;  // exact: below 2^24
            return FZ_OK;
        }
        default: return FZ_ERR_ARG;
    }
}

}  // namespace fz

extern "C" {

size_t fz_compress_bound(const fz_dims* dims)
{
    Geom g;
    if (!geom_of(dims, &g)) return 0;
    return (size_t)g.bound;
}

size_t fz_header_bytes(const fz_dims* dims)
{
    Geom g;
    if (!geom_of(dims, &g)) return 0;
    return (size_t)g.payload_off;
}

size_t fz_stream_bound(const fz_dims* dims)
{
    Geom g;
    if (!geom_of(dims, &g)) return 0;
    return (size_t)g.stream_bound;
}

int fz_compress_timed(const float* d_in, const fz_dims* dims, double eb, int eb_mode, void* d_out, void* stream,
                      const fz_timing* timing)
{
    Geom g;
    if (!d_in || !d_out || !geom_of(dims, &g) || !aligned_to(d_in, 4) || !aligned_to(d_out, 256)) return FZ_ERR_ARG;
    float ebx2 = 0.0f, inv = 0.0f;
    const int rc = bound_params(eb, eb_mode, &ebx2, &inv);
    if (rc != FZ_OK) return rc;
    const HeaderImage h = header_image(g, eb, eb_mode, ebx2, inv);
    Timing t{};
    if (timing) {
        t.range_begin = static_cast<hipEvent_t>(timing->range_begin);
        t.main_begin = static_cast<hipEvent_t>(timing->main_begin);
        t.main_end = static_cast<hipEvent_t>(timing->main_end);
        t.done = static_cast<hipEvent_t>(timing->done);
    }
    uint8_t* out = static_cast<uint8_t*>(d_out);
    hipError_t e = launch_compress(d_in, out, out + g.scratch_off, g, h, eb_mode, eb, static_cast<hipStream_t>(stream),
                                   timing ? &t : nullptr);
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_compress(const float* d_in, const fz_dims* dims, double eb, int eb_mode, void* d_out, void* stream)
{
    return fz_compress_timed(d_in, dims, eb, eb_mode, d_out, stream, nullptr);
}

// the checks every decompression entry point makes on its arguments
static bool decompress_args(const void* d_stream, size_t stream_bytes, const void* d_out, size_t align_out,
                            const fz_dims* dims, const uint32_t* d_err, Geom* g)
{
    return d_stream && d_out && geom_of(dims, g) && aligned_to(d_stream, 256) && aligned_to(d_out, align_out) &&
           aligned_to(d_err, 4) && stream_bytes >= (size_t)g->payload_off;
}

int fz_decompress(const void* d_stream, size_t stream_bytes, float* d_out, const fz_dims* dims, uint32_t* d_err,
                  void* stream)
{
    Geom g;
    if (!decompress_args(d_stream, stream_bytes, d_out, 4, dims, d_err, &g)) return FZ_ERR_ARG;
    hipError_t e = launch_decompress(static_cast<const uint8_t*>(d_stream), stream_bytes, d_out, g, d_err,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

size_t fz_compress_bound_f64(const fz_dims* dims)
{
    Geom g;
    if (!geom_of(dims, &g)) return 0;
    return (size_t)g.bound64;
}

int fz_compress_f64(const double* d_in, const fz_dims* dims, double eb, int eb_mode, void* d_out, void* stream)
{
    Geom g;
    if (!d_in || !d_out || !geom_of(dims, &g) || !aligned_to(d_in, 8) || !aligned_to(d_out, 256)) return FZ_ERR_ARG;
    if (!(eb > 0.0) || !std::isfinite(eb) || (eb_mode != FZ_EB_ABS && eb_mode != FZ_EB_REL)) return FZ_ERR_ARG;
    double ebx2 = 0.0, inv = 0.0;  // REL: derived on the device
    if (eb_mode == FZ_EB_ABS) {
        ebx2 = 2.0 * eb;
        inv = 1.0 / ebx2;
        if (!(ebx2 >= DBL_MIN) || !std::isfinite(ebx2) || !std::isfinite(inv) || !(inv > 0.0)) return FZ_ERR_EB_RANGE;
    }
    const HeaderImage h = header_image_f64(g, eb, eb_mode, ebx2, inv);
    hipError_t e = launch_compress_f64(d_in, static_cast<uint8_t*>(d_out), g, h, eb_mode, eb,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_decompress_f64(const void* d_stream, size_t stream_bytes, double* d_out, const fz_dims* dims, uint32_t* d_err,
                      void* stream)
{
    Geom g;
    if (!decompress_args(d_stream, stream_bytes, d_out, 8, dims, d_err, &g)) return FZ_ERR_ARG;
    hipError_t e = launch_decompress_f64(static_cast<const uint8_t*>(d_stream), stream_bytes, d_out, g, d_err,
                                         static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

size_t fz_compress_bound_global(const fz_dims* dims)
{
    Geom g;
    if (!geom_of(dims, &g)) return 0;
    return (size_t)g.bound64;  // the fp32 bound, then the integers the chunk kernel reads
}

int fz_compress_global(const float* d_in, const fz_dims* dims, double eb, int eb_mode, void* d_out, void* stream)
{
    Geom g;
    if (!d_in || !d_out || !geom_of(dims, &g) || !aligned_to(d_in, 4) || !aligned_to(d_out, 256)) return FZ_ERR_ARG;
    float ebx2 = 0.0f, inv = 0.0f;
    const int rc = bound_params(eb, eb_mode, &ebx2, &inv);
    if (rc != FZ_OK) return rc;
    HeaderImage h = header_image(g, eb, eb_mode, ebx2, inv);
    const uint8_t global = 1;
    put_bytes(h, kOffPredictor, &global, 1);
    hipError_t e = launch_compress_global(d_in, static_cast<uint8_t*>(d_out), g, h, eb_mode, eb,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

size_t fz_decompress_global_work_bytes(const fz_dims* dims)
{
    Geom g;
    if (!geom_of(dims, &g)) return 0;
    return global_work_bytes(g);
}

int fz_decompress_global(const void* d_stream, size_t stream_bytes, float* d_out, const fz_dims* dims,
                         uint32_t* d_err, void* d_work, void* stream)
{
    Geom g;
    if (!decompress_args(d_stream, stream_bytes, d_out, 4, dims, d_err, &g) || !d_work || !aligned_to(d_work, 256))
        return FZ_ERR_ARG;
    hipError_t e = launch_decompress_global(static_cast<const uint8_t*>(d_stream), stream_bytes, d_out, g, d_err,
                                            d_work, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FZ_OK : FZ_ERR_HIP;
}

int fz_stream_info(const void* h_header, size_t n, fz_info* out)
{
    if (!h_header || !out || n < (size_t)kHeaderBytes) return FZ_ERR_ARG;
    const uint8_t* s = static_cast<const uint8_t*>(h_header);
    uint32_t magic;
    uint16_t ver, hb;
    std::memcpy(&magic, s + kOffMagic, 4);
    std::memcpy(&ver, s + kOffVersion, 2);
    std::memcpy(&hb, s + kOffHdrBytes, 2);
    if (magic != kMagic) return FZ_ERR_STREAM;
    if (ver != kVersion || hb != kHeaderBytes) return FZ_ERR_VERSION;
    std::memset(out, 0, sizeof(*out));
    out->version = ver;
    std::memcpy(&out->status, s + kOffStatus, 4);
    out->rank = s[kOffRank];
    out->eb_mode = s[kOffEbMode];
    std::memcpy(out->n, s + kOffDims, 24);
    std::memcpy(&out->eb_user, s + kOffEbUser, 8);
    std::memcpy(&out->ebx2, s + kOffEbx2, 4);
    std::memcpy(&out->inv, s + kOffInv, 4);
    std::memcpy(&out->vmin, s + kOffVmin, 4);
    std::memcpy(&out->vmax, s + kOffVmax, 4);
    std::memcpy(&out->n_chunks, s + kOffNChunks, 4);
    std::memcpy(&out->nnz_blocks, s + kOffNnz, 8);
    std::memcpy(&out->n_outliers, s + kOffNout, 8);
    std::memcpy(&out->total_bytes, s + kOffTotal, 8);
    Geom g;
    if (make_geom((int)out->rank, out->n, &g)) out->header_bytes = (uint64_t)g.payload_off;
    out->dtype = s[kOffDtype];
    out->predictor = s[kOffPredictor];
    std::memcpy(&out->ebx2_f64, s + kOffEbx2F64, 8);
    std::memcpy(&out->inv_f64, s + kOffInvF64, 8);
    return FZ_OK;
}

const char* fz_strerror(int status)
{
    switch (status) {
        case FZ_OK: return "ok";
        case FZ_ERR_ARG: return "invalid argument";
        case FZ_ERR_HIP: return "HIP runtime error";
        case FZ_ERR_NONFINITE: return "input holds NaN or Inf";
        case FZ_ERR_EB_RANGE: return "error bound out of range";
        case FZ_ERR_OUTLIER_CAP: return "too many escaped codes";
        case FZ_ERR_STREAM: return "malformed stream";
        case FZ_ERR_VERSION: return "unsupported stream version";
        case FZ_ERR_STATUS: return "stream carries a compression error";
        default: return "unknown status";
    }
}

}  // extern "C"
