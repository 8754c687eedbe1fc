// Launch interface between the C ABI and the decode kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "csgv_format.h"

namespace csgv {

// Per work-group scratch (global memory): decoded rANS symbols, then the
// level grids and parent list of bricks decoded outside LDS.
constexpr uint64_t kScratchSymBytes = ((8 * total_nodes(kMaxLog2b) + 64 + 255) / 256) * 256;
constexpr uint64_t kBigOddSlots = 1u << 15;   // levels 1, 3, 5
constexpr uint64_t kBigEvenSlots = 1u << 18;  // levels 0, 2, 4, 6
constexpr uint64_t kBigListBytes = (1u << 15) * 2;
constexpr uint64_t kScratchPerWG = kScratchSymBytes + 4 * (kBigOddSlots + kBigEvenSlots) + kBigListBytes;

struct Params {
    const uint8_t* vol;  // container in device memory
    uint64_t vol_bytes;
    uint64_t off_pos;
    uint32_t n_bricks;
    uint32_t label_bytes;
    uint32_t freq_ok;
    uint32_t freq[8];  // 16 x u16
    const uint32_t* ids;
    const uint8_t* lods;
    const uint64_t* out_offs;
    uint32_t n_tasks;
    uint32_t task0;     // first task of a non-queue launch
    uint8_t* out;
    uint64_t out_cap;   // elements
    uint32_t* status;   // may be null
    uint32_t* queue;    // persistent form: next-task counter (null otherwise)
    const uint32_t* order;  // optional pop order
    uint8_t* scratch;
    uint64_t scratch_stride;
};

size_t shared_bytes();
hipError_t set_kernel_attrs();
hipError_t launch_decode(const Params& P, int wg_size, uint32_t grid, hipStream_t s);
hipError_t launch_reset(uint32_t* q, hipStream_t s);
hipError_t launch_sort(const Params& P, uint32_t* cls, uint32_t* hist, uint32_t* order, hipStream_t s);

}  // namespace csgv
