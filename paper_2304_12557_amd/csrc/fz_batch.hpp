// fz_batch.hpp -- internal: batch plans of libfzmi (host side), shared by the
// batch entry points (fz_batch.hip) and the request server (fz_server.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "fz.h"
#include "fz_format.hpp"
#include "fz_kernels.hpp"

namespace fz {

struct CompressJob {
    const float* x;
    uint8_t* out;
    Geom g;
    HeaderImage h;
    double eb;
    int32_t key;  // rank * 2 + (16-byte aligned rows ? 1 : 0)
    int32_t rel;
    int64_t chunk0;     // first ticket of this field in its class's part of the chunk table
    int64_t chunkg;     // first entry of this field in the whole chunk table
    int64_t mm0;        // first range-pass block of this field (REL)
    int64_t mm_blocks;  // range-pass blocks of this field (REL)
};

struct DecompressJob {
    const uint8_t* s;
    float* y;
    Geom g;
    uint32_t* err;
    int32_t key;
    int32_t pad;
    int64_t chunk0;
    uint64_t s_bytes;  // bytes readable at s
};

struct Tuning {
    int per_cu;  // persistent compression workgroups per CU (1 or 2)
    int mm_cap;  // range-pass blocks per field, at most
};

// compute units of the current device (1 if unknown)
int cu_count();

// staging slots of a compression plan (one per persistent workgroup) and
// their bytes, for a device with `cus` compute units
inline int stage_slots(int cus) { return 2 * cus < kStageSlots ? 2 * cus : kStageSlots; }
inline size_t stage_bytes(int cus) { return (size_t)stage_slots(cus) * (size_t)kStageSlotBytes; }

struct Plan {
    bool compress;
    int n_jobs;
    int64_t total_chunks;
    int64_t class_off[8], class_chunks[8];  // compression: the chunk table is ordered by class (key)
    int64_t total_mm;
    int64_t mm_max;  // range-pass blocks with the largest per-field cap
    bool any_rel;
    int cus;
    Tuning tune;
    std::vector<CompressJob> cjobs;
    std::vector<DecompressJob> djobs;
    void* dev;  // device block of a standalone plan: ticket, job table, chunk -> job, block -> job
    size_t off_jobs, off_chunk, off_mm;
    uint32_t* d_ticket;
    void* d_jobs;
    int32_t* d_chunk_job;
    int32_t* d_mm_job;
    void* d_stage;  // compression: stage_bytes(cus) of staging slots (the plan's own, or its server slot's)
};

// Build a plan from jobs on the host (validates them; no device work).
int plan_compress(Plan* P, int n, const fz_compress_job* jobs);
int plan_decompress(Plan* P, int n, const fz_decompress_job* jobs);
// Host image of the plan's device tables for its current tuning; returns its
// size (with room for cap_mm range-pass block entries).
size_t plan_layout(Plan* P, int64_t cap_mm, std::vector<uint8_t>* img);
// Point the plan at the device area holding its image.
void plan_bind(Plan* P, void* dev);
// Enqueue the plan's kernels on a stream.
hipError_t plan_run(const Plan* P, hipStream_t st);

}  // namespace fz
