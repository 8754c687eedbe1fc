// Launch interface between the C ABI and the decode kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "csgv_format.h"

namespace csgv {

// ---- LDS of a decode work-group: a fixed part plus `cap16` 16-bit slots for
// the explicit nodes of level 5 (the LDS split chosen per launch).  The slot
// area also holds the 16 KiB rANS decoding table while a record's symbols are
// decoded, so it is never smaller than kMinCap16 slots.
constexpr uint32_t kMaxWaves = 16;       // work-groups of up to 1024 threads
constexpr uint32_t kFullSlots = 4688;    // full grids of levels 0..4 at 0, 8, 16, 80, 592
constexpr uint32_t kEWords = 148;        // expansion bitmaps of levels 0..4: 1+1+2+16+128 words
constexpr uint32_t kUBytes = 8192;       // parent list of the level being decoded | staged palette
constexpr uint32_t kMinCap16 = 8192;     // 16 KiB: the rANS table
constexpr uint32_t kMaxCap16 = 32760;    // largest LDS slot share accepted
constexpr uint32_t kDefaultCap16 = 10240;

// ---- per work-group global scratch (byte offsets).  Big-path level storage
// (32-bit slots: full grids of levels 0..4, level 5 by rank), the level-5
// bitmap used by 64^3 bricks, parent lists of level 6 (and of every level on
// the big path), then the decoded rANS symbols (4 bits each) whose size
// depends on the largest brick side of the volume.
constexpr uint64_t kScrFull = 0;                                   // 4688 x u32
constexpr uint64_t kScrComp = 18944;                               // 32768 x u32
constexpr uint64_t kScrE5 = kScrComp + 4ull * 32768;               // 1024 x u32
constexpr uint64_t kScrWpre5 = kScrE5 + 4096;                      // 1024 x u16
constexpr uint64_t kScrList = kScrWpre5 + 2048;                    // 32768 x u16
constexpr uint64_t kScrPval = kScrList + 65536;                    // 32768 x u32
constexpr uint64_t kScrSym = kScrPval + 131072;                    // 4-bit symbols
constexpr uint64_t scratch_per_wg(uint32_t max_log2b) {
    return kScrSym + ((4 * total_nodes(max_log2b) + 255) / 256) * 256;
}

struct RansFreq {
    uint32_t w[8];  // 16 x u16 frequencies, two per word
};

struct Params {
    const uint8_t* vol;  // container in device memory
    uint64_t vol_bytes;
    uint64_t off_pos;
    uint32_t n_bricks;
    uint32_t label_bytes;
    uint32_t freq_ok;          // the volume's frequency table sums to 4096
    uint32_t max_log2b;        // records with a larger brick side are rejected (scratch bound)
    const uint32_t* rans_tab;  // decoding table built by rans_table_kernel (4096 entries)
    const uint32_t* ids;
    const uint8_t* lods;
    const uint64_t* out_offs;    // caller's element offsets, or null
    const uint64_t* dense_offs;  // offsets computed on the device when out_offs is null
    uint32_t n_tasks;
    uint32_t task0;     // first task of a non-queue launch
    uint8_t* out;
    uint64_t out_cap;   // elements
    uint32_t* status;   // may be null
    uint32_t* queue;    // persistent form: next-task counter (null otherwise)
    const uint32_t* order;  // optional pop order
    uint8_t* scratch;
    uint64_t scratch_stride;
    uint32_t cap16;     // LDS slots for the explicit nodes of level 5 (>= kMinCap16)
    uint32_t pal_bits;  // 0: labels; I > 0: packed I-bit palette indices, floor(32/I) per word
};

// output units of an S^3 cube: labels, or 32-bit words of packed palette indices
__host__ __device__ inline uint64_t out_units(uint64_t voxels, uint32_t pal_bits) {
    if (!pal_bits) return voxels;
    const uint64_t e = 32u / pal_bits;
    return (voxels + e - 1) / e;
}

size_t shared_bytes(uint32_t cap16);
int max_resident_per_cu(int wg_size, uint32_t cap16);  // occupancy of the decode kernel
hipError_t set_kernel_attrs();
hipError_t launch_decode(const Params& P, int wg_size, uint32_t grid, hipStream_t s);
hipError_t launch_reset(uint32_t* q, hipStream_t s);
hipError_t launch_rans_table(uint32_t* tab, const RansFreq& f, hipStream_t s);
hipError_t launch_sort(const Params& P, uint32_t* cls, uint32_t* hist, uint32_t* order, hipStream_t s);
hipError_t launch_dense_offsets(const Params& P, uint64_t* offs, hipStream_t s);

}  // namespace csgv
