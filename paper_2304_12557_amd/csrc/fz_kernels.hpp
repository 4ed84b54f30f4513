// fz_kernels.hpp -- internal launchers of libfzmi (host side of the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include "fz_format.hpp"

namespace fz {

struct HeaderImage {
    uint32_t w[kHeaderBytes / 4];
};

hipError_t launch_compress(const float* x, uint8_t* out, const Geom& g, const HeaderImage& h, bool rel, double eb,
                           hipStream_t st);
hipError_t launch_decompress(const uint8_t* s, float* y, const Geom& g, uint32_t* d_err, hipStream_t st);

}  // namespace fz
