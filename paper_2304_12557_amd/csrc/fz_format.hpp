// fz_format.hpp -- stream format v1 constants and chunk geometry (device +
// host side of libfzmi).
//
// Stream layout (little-endian):
//   header (128 B) | chunk table (8 B per chunk, padded to 16 B) |
//   flags (512 B per chunk) | payload (16-B units)
// A chunk is the unit of independent decompression: the Lorenzo predictor
// (Sec. 2.3) runs inside its box with zero ghosts at the box faces.  Boxes
// (slowest-first): 3-D 16 x 32 x 64, 2-D 32 x 1024, 1-D 32768 values.
// A chunk holds up to 16 steps of 2048 codes (64 patches of 32 codes), and
// 4 steps form a layer.  The data block of the zero-block encoder (Sec. 3.4)
// is a brick: one bit plane of one patch over the 4 steps of a layer
// (128 bits), i.e. the bitshuffle of Sec. 3.3 gathers bit b of 128 codes that
// are neighbours in space (3-D: a 4x4x8 box; 2-D: 8x16; 1-D: 4 runs of 32).
//   code index n = step*2048 + patch*32 + cell
//   3-D: z = step, y = 4*(patch%8) + cell/8, x = 8*(patch/8) + cell%8
//   2-D: y = 2*step + cell/16, x = 16*patch + cell%16
//   1-D: x = 2048*step + 32*patch + cell
//   brick (layer k, plane b, patch p): bit 32*t + m = bit b of code
//   (4k+t, p, m); flags of layer k: 16 u64 words, bit p of word b = brick
//   nonzero; payload of a chunk: nonzero bricks in (k, b, p) order, then the
//   escape pairs {u32 n, i32 delta} ascending in n, padded to 16 B.
#pragma once
#include <stdint.h>

namespace fz {

constexpr uint32_t kMagic = 0x314D5A46u;  // "FZM1"
constexpr uint16_t kVersion = 1;
constexpr int kHeaderBytes = 128;
constexpr int kSteps = 16;
constexpr int kStepCodes = 2048;
constexpr int kPatches = 64;
constexpr int kPatchCodes = 32;
constexpr int kLayers = 4;
constexpr int kPlanes = 16;
constexpr int kChunkCodes = kSteps * kStepCodes;
constexpr int kFlagBytesPerChunk = kLayers * kPlanes * 8;
// escapes a chunk may store: 1/32 of its codes (the worst-case payload of a
// chunk, which sizes the bound, counts this many pairs)
constexpr int kChunkOutlierCap = 1024;
constexpr uint32_t kEscape = 0x8000u;
// worst-case payload of one chunk: every brick nonzero plus the escape cap
constexpr int64_t kChunkPayloadBound = (int64_t)kLayers * kPlanes * kPatches * 16 + kChunkOutlierCap * 8;

// header byte offsets
constexpr int kOffMagic = 0, kOffVersion = 4, kOffHdrBytes = 6, kOffStatus = 8, kOffDtype = 12, kOffRank = 13,
              kOffEbMode = 14, kOffDims = 16, kOffEbUser = 40, kOffEbx2 = 48, kOffInv = 52, kOffVmin = 56,
              kOffVmax = 60, kOffChunk = 64, kOffNChunks = 72, kOffNnz = 80, kOffNout = 88, kOffTotal = 96;
// fp64 streams (dtype 1): 2 eb_abs and its reciprocal as doubles (zero in fp32 streams)
constexpr int kOffEbx2F64 = 104, kOffInvF64 = 112;
// byte 15: the Lorenzo predictor, 0 inside each chunk, 1 over the whole field
constexpr int kOffPredictor = 15;

// status bits
constexpr uint32_t kErrNonfinite = 1u, kErrEbRange = 2u, kErrOutlierCap = 4u;
constexpr uint32_t kErrInternal = 0x80000000u;  // a consistency check of the library failed

// scratch (after the worst-case stream) used by one compression
struct Scratch {
    uint32_t ticket;      // chunk tickets, in launch order
    uint32_t pre_status;  // errors found before the main pass (REL params)
    uint32_t done;        // compression workgroups that have finished
    uint32_t pad[13];
    // followed by a copy of the Geom at byte 64 (read by out-of-line device
    // code) and by uint64_t state[n_chunks] at byte kScratchStateOff
};
constexpr int kScratchGeomOff = 64;
constexpr int kScratchStateOff = 512;
// per-block partial value ranges of the REL pass, after the chunk states
constexpr int kMinmaxBlocks = 2048;
// staging: each compression workgroup assembles a chunk's compacted payload
// in a slot of its own (at scr_stage + workgroup * slot bytes in the scratch)
// and copies it to its place in the stream once the chunk's offset is known;
// the grid has at most kStageSlots workgroups
constexpr int64_t kStageSlotBytes = kChunkPayloadBound;
constexpr int kStageSlots = 768;

// chunk state word: flag in the top 2 bits, value below.  A chunk publishes
// its payload size in 16-B units (kFlagAgg) once its layers are coded, and
// its inclusive prefix (kFlagIncl) once its offset is known
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagIncl = 2ull << 62, kValueMask = (1ull << 62) - 1;

struct Geom {  // kept trivially copyable and below 448 bytes (it is copied into the scratch)
    int rank;
    int box[3];
    int64_t n[3];     // slowest-first, trailing unused = 1
    int64_t grid[3];  // chunks per dimension
    int64_t n_chunks;
    int64_t table_off, flags_off, payload_off;  // = header bytes
    int64_t stream_bound;  // worst-case stream bytes
    // scratch of one compression: at scratch_off in the output buffer (right
    // after the worst-case stream), or in a buffer of its own; scr_minmax and
    // scr_stage are offsets inside it, scr_bytes its size
    int64_t scratch_off, scr_minmax, scr_stage, scr_bytes;
    int64_t bound;  // the output buffer with its scratch: scratch_off + scr_bytes
    // fp64 input: the prequantized integers (4 B per value) and the partial
    // value ranges of its REL pass follow the fp32 bound
    int64_t q_off, part64_off, bound64;
};
// per-block partials of the fp64 range pass: min and max (2 doubles), then a
// u32 non-finite flag per block after all the doubles
constexpr int64_t kPart64Bytes = 20 * kMinmaxBlocks;

// whether p is a multiple of a (a power of two); null counts as aligned
inline bool aligned_to(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

inline bool make_geom(int rank, const uint64_t* dims, Geom* g)
{
    if (rank < 1 || rank > 3) return false;
    g->rank = rank;
    for (int i = 0; i < 3; i++) { g->n[i] = 1; g->box[i] = 1; }
    for (int i = 0; i < rank; i++) {
        if (dims[i] == 0 || dims[i] > (1ull << 40)) return false;
        g->n[i] = (int64_t)dims[i];
    }
    // the contiguous extent of a 2-D/3-D field stays below 2^25 so that lane
    // offsets inside one step fit in 32 bits
    if (rank >= 2 && dims[rank - 1] >= (1ull << 25)) return false;
    if (rank == 3) { g->box[0] = 16; g->box[1] = 32; g->box[2] = 64; }
    if (rank == 2) { g->box[0] = 32; g->box[1] = 1024; }
    if (rank == 1) { g->box[0] = 32768; }
    g->n_chunks = 1;
    for (int i = 0; i < 3; i++) {
        g->grid[i] = (g->n[i] + g->box[i] - 1) / g->box[i];
        g->n_chunks *= g->grid[i];
    }
    if (g->n_chunks >= (1ll << 31)) return false;
    int64_t table = (8 * g->n_chunks + 15) / 16 * 16;
    g->table_off = kHeaderBytes;
    g->flags_off = kHeaderBytes + table;
    g->payload_off = g->flags_off + (int64_t)kFlagBytesPerChunk * g->n_chunks;
    g->stream_bound = g->payload_off + g->n_chunks * kChunkPayloadBound;
    g->scratch_off = (g->stream_bound + 255) / 256 * 256;
    g->scr_minmax = kScratchStateOff + 8 * g->n_chunks;
    g->scr_stage = (g->scr_minmax + 16 * kMinmaxBlocks + 255) / 256 * 256;
    g->scr_bytes = g->scr_stage + (g->n_chunks < kStageSlots ? g->n_chunks : kStageSlots) * kStageSlotBytes;
    g->bound = g->scratch_off + g->scr_bytes;
    const int64_t n = g->n[0] * g->n[1] * g->n[2];  // below 2^46: fewer than 2^31 chunks of 2^15 values
    g->q_off = (g->bound + 255) / 256 * 256;
    g->part64_off = g->q_off + (4 * n + 255) / 256 * 256;
    g->bound64 = g->part64_off + kPart64Bytes;
    return true;
}

}  // namespace fz
