// Byte layout of the CSGV container as read by the GPU decoder and written by
// the host encoder.  (The CPU oracle keeps its own copy of these constants.)
#pragma once
#include <stdint.h>

namespace csgv {

constexpr uint32_t kMagic = 0x56475343u;  // 'CSGV'
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 128;

// header field offsets
constexpr uint32_t kHdrDims = 8, kHdrLog2b = 20, kHdrLabelBytes = 24, kHdrOpMask = 28, kHdrNBricks = 32,
                   kHdrGrid = 36, kHdrFreq = 48, kHdrOffsetsPos = 80, kHdrDirPos = 88, kHdrTotal = 96,
                   kHdrNeighborMode = 104;

// operation codes (low 3 bits of a symbol; bit 3 is the stop bit)
enum Op : uint32_t { kParent = 0, kNX = 1, kNY = 2, kNZ = 3, kAdv = 4, kLast = 5, kDelta = 6, kBadOp = 7 };

// per-task status
enum TaskStatus : uint32_t { kTaskOk = 0, kTaskInvalid = 1, kTaskCorrupt = 2 };

enum Coder : uint32_t { kRaw4 = 0, kRans = 1 };

constexpr uint32_t kMaxLog2b = 6;
constexpr uint32_t kRansBits = 12, kRansM = 1u << kRansBits, kRansL = 1u << 16;

// nodes of levels 0..L together: (8^(L+1) - 1) / 7
constexpr uint64_t total_nodes(uint32_t L) { return ((uint64_t(1) << (3 * (L + 1))) - 1) / 7; }

// bytes of the fixed record header for a brick of side 2^L
constexpr uint64_t record_header_bytes(uint32_t L, uint32_t coder, uint32_t log2W) {
    return 8 + 4ull * (L + 1) + (coder == kRans ? 4ull * (((1u << log2W) + 63) / 64) + 4ull * (1u << log2W) : 0);
}

}  // namespace csgv
