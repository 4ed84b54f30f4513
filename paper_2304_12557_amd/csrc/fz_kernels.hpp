// fz_kernels.hpp -- internal launchers of libfzmi (host side of the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include "fz_format.hpp"

namespace fz {

struct HeaderImage {
    uint32_t w[kHeaderBytes / 4];
};

// events recorded between the launches of one compression (each may be null)
struct Timing {
    hipEvent_t range_begin, main_begin, main_end, done;
};

// mode: FZ_EB_ABS, FZ_EB_REL (adds the range pass) or FZ_EB_PWREL; the
// compression's scratch (g.scr_bytes) at scr: out + g.scratch_off, or a
// buffer of its own
hipError_t launch_compress(const float* x, uint8_t* out, uint8_t* scr, const Geom& g, const HeaderImage& h, int mode,
                           double eb, hipStream_t st, const Timing* t = nullptr);
// decompression: sb = the bytes readable at s (at least g.payload_off,
// checked by the caller); no byte past them is read
hipError_t launch_decompress(const uint8_t* s, uint64_t sb, float* y, const Geom& g, uint32_t* d_err, hipStream_t st);
// fp64 input (FZ_EB_ABS or FZ_EB_REL): the range pass (REL) and the
// prequantization into the integer buffer at g.q_off, then the compression
// kernel on those integers
hipError_t launch_compress_f64(const double* x, uint8_t* out, const Geom& g, const HeaderImage& h, int mode,
                               double eb, hipStream_t st);
hipError_t launch_f64_front(const double* x, uint8_t* out, const Geom& g, int mode, double eb, hipStream_t st);
hipError_t launch_decompress_f64(const uint8_t* s, uint64_t sb, double* y, const Geom& g, uint32_t* d_err,
                                 hipStream_t st);
// copy the header's status to the scratch's pre_status (after a pass that
// wrote the integer buffer)
hipError_t launch_pre_status(uint8_t* out, const Geom& g, hipStream_t st);
// field-global Lorenzo predictor: compression (any fp32 mode) and
// decompression with its carry passes, which need global_work_bytes(g) of
// device memory at `work`
hipError_t launch_compress_global(const float* x, uint8_t* out, const Geom& g, const HeaderImage& h, int mode,
                                  double eb, hipStream_t st);
hipError_t launch_face(const float* x, uint8_t* out, const Geom& g, hipStream_t st);
hipError_t launch_decompress_global(const uint8_t* s, uint64_t sb, float* y, const Geom& g, uint32_t* d_err,
                                    void* work, hipStream_t st);
size_t global_work_bytes(const Geom& g);

// whether compression may read a field at x with 16-byte loads (4-byte aligned values)
bool vec_loads(const void* x);
// blocks of the REL range pass of a field of n values
int64_t minmax_blocks(int64_t n);
// header image of a stream (magic, version, dims, eb, chunk box, ...)
HeaderImage header_image(const Geom& g, double eb, int mode, float ebx2, float inv);
// the same for an fp64 stream (dtype 1; the double parameters at their own offsets)
HeaderImage header_image_f64(const Geom& g, double eb, int mode, double ebx2, double inv);
// eb parameters of an absolute bound; false if unusable
bool abs_params(double eb, float* ebx2, float* inv);
// the header's quantizer fields for a bound and mode, as far as the host
// knows them (REL: derived on the device, 0 here; PWREL: ebx2 holds the step
// S = floor(eb * 2^24 / (1 + eb)), inv 0).  Returns FZ_OK, FZ_ERR_ARG (eb not
// finite and > 0, unknown mode) or FZ_ERR_EB_RANGE (unusable bound).
int bound_params(double eb, int mode, float* ebx2, float* inv);

}  // namespace fz
