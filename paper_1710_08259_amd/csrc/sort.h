// Stable LSD radix sort of (key, value) pairs of 32-bit words on gfx950.
//
// The cell list orders particles by cell key (Sec. 3.2.1): one stable sort
// of (key, original index) serves every case of a batch.
#pragma once

#include "internal.h"

namespace nau {

constexpr uint32_t kSortTile = 4096;  // keys per workgroup in the histogram and scatter passes
constexpr uint32_t kSortBins = 256;   // digits of at most 8 bits

// Number of digit passes for keys of `bits` bits (passes of at most 8 bits,
// balanced).  The sorted pairs land in buffer (passes % 2) of the ping-pong
// pair below.
__host__ __device__ inline int radix_passes(int bits) { return (bits + 7) / 8; }

// Sorts the n pairs (keys[0][i], vals[0][i]) by the low `bits` bits of the
// key, stably, ping-ponging between buffers 0 and 1; the result is in buffer
// radix_passes(bits) % 2.  hist holds kSortBins * ceil(n / kSortTile) words,
// totals kSortBins words.  Keys must be below 2^bits.  `ordered` orders each
// tile by digit in LDS before its stores: a gain where consecutive keys
// mostly differ (fewer keys than cells), a loss where they share cells.
hipError_t launch_radix_sort(uint32_t* const keys[2], uint32_t* const vals[2], uint32_t n, int bits,
                             bool ordered, uint32_t* hist, uint32_t* totals, hipStream_t s);

}  // namespace nau
