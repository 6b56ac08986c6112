// Neighbour-list entries: one 32-bit word per pair, the neighbour index in the low 22
// bits and the periodic image (shifts sx, sy, sz in box lengths) in three 3-bit fields
// stored with an offset of 3, so each shift may be -3 .. 4.  The pair searches only
// produce shifts in -3 .. 3: the parameter rules keep the real-space reach (cutoff times
// sqrt(1 + gamma^2) on a sheared lattice, |gamma| <= 1/2) below three box lengths.
#pragma once
#include <cstdint>

namespace fsd {

constexpr int kPairIndexBits = 22;
constexpr uint32_t kPairIndexMask = (1u << kPairIndexBits) - 1u;

__host__ __device__ inline uint32_t pack_entry(int j, int sx, int sy, int sz) {
  return uint32_t(j) | (uint32_t(sx + 3) << 22) | (uint32_t(sy + 3) << 25) | (uint32_t(sz + 3) << 28);
}

__host__ __device__ inline int entry_index(uint32_t c) { return int(c & kPairIndexMask); }

// image shift along axis 0 (x), 1 (y) or 2 (z)
__host__ __device__ inline int entry_shift(uint32_t c, int axis) { return int((c >> (22 + 3 * axis)) & 7u) - 3; }

}  // namespace fsd
