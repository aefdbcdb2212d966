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
// ---- one tile in one workgroup --------------------------------------------------
// A table of at most kSortTile keys is sorted by one workgroup of
// kTileThreads threads with every digit pass in LDS.  Keys ping-pong between
// key[0] and key[1], each with its place in the input (16 bits) in idx[].
// Wave w owns the contiguous chunk [w * 256, (w + 1) * 256) of each pass's
// input, in four rows of 64.  A pass ranks every key within its row (wave
// ballots) and against the earlier rows of its chunk (a count per digit
// private to the wave), then one step per digit turns the waves' counts
// into where each wave's keys of that digit start, and each wave scatters
// its chunk.  Input order is (wave, row, lane), so the sort is stable; a
// pass takes four barriers.
constexpr int kTileThreads = 1024;
constexpr int kTileWaves = kTileThreads / kWave;
constexpr int kTileIters = static_cast<int>(kSortTile) / kTileThreads;
constexpr uint32_t kTileChunk = kSortTile / kTileWaves;  // keys per wave
constexpr int kTileRows = static_cast<int>(kTileChunk) / kWave;
static_assert(kTileIters * kTileThreads == static_cast<int>(kSortTile), "a tile is a whole number of rows");
static_assert(kTileRows * kWave * kTileWaves == static_cast<int>(kSortTile), "a chunk is a whole number of rows");
static_assert(kSortTile <= 65535u, "places and counts are 16-bit");

struct TileSort {
    uint32_t key[2][kSortTile];
    uint16_t idx[2][kSortTile];
    uint16_t cnt[kTileWaves][kSortBins];  // per wave and digit: a count, then where the wave's keys go
    uint32_t tmp[kSortBins / kWave];
};

// Sorts key[0][0 .. n) (with idx[0][0 .. n) their places) by the low `bits`
// bits, stably; returns the buffer the result is in.  Every thread of the
// workgroup calls it after filling key[0] and idx[0]; the result is visible
// to all threads on return.
__device__ inline int tile_sort(TileSort& sm, uint32_t n, int bits)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t wave = tid / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int passes = radix_passes(bits);
    const int per = (bits + passes - 1) / passes;
    int src = 0;
    __syncthreads();  // the caller's fill
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * per;
        const int b = (bits - shift) < per ? (bits - shift) : per;
        const uint32_t bins = 1u << b;
        const uint32_t mask = bins - 1u;
        for (uint32_t d = lane; d < bins; d += kWave) sm.cnt[wave][d] = 0;
        // rank each key among the keys of its digit before it in this chunk
        uint32_t dig[kTileRows], before[kTileRows], kv[kTileRows];
        uint16_t iv[kTileRows];
        bool val[kTileRows];
#pragma unroll
        for (int r = 0; r < kTileRows; ++r) {
            const uint32_t i = wave * kTileChunk + r * kWave + lane;
            val[r] = i < n;
            kv[r] = val[r] ? sm.key[src][i] : 0u;
            iv[r] = val[r] ? sm.idx[src][i] : uint16_t{0};
            const uint32_t d = (kv[r] >> shift) & mask;
            uint64_t peers = __ballot(val[r]);
            for (int bb = 0; bb < b; ++bb) {
                const bool bit = (d >> bb) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t rank = __popcll(peers & lt_mask);
            const uint32_t so_far = sm.cnt[wave][d];  // every lane of the digit reads it ...
            if (val[r] && rank == 0) sm.cnt[wave][d] = static_cast<uint16_t>(so_far + __popcll(peers));  // ... then one adds
            dig[r] = d;
            before[r] = so_far + rank;
        }
        __syncthreads();
        // per digit: each wave's start among the digit's keys (waves in
        // order), and the digit's start among all keys (digits in order)
        uint32_t total = 0, inc = 0;
        uint32_t c[kTileWaves];
        if (tid < kSortBins) {
#pragma unroll
            for (int w = 0; w < kTileWaves; ++w) {
                c[w] = tid < bins ? sm.cnt[w][tid] : 0u;
                total += c[w];
            }
            inc = total;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t o = __shfl_up(inc, d, kWave);
                if (lane >= static_cast<uint32_t>(d)) inc += o;
            }
            if (lane == kWave - 1) sm.tmp[wave] = inc;
        }
        __syncthreads();
        if (tid < bins) {
            uint32_t at = inc - total;
            for (uint32_t w = 0; w < wave; ++w) at += sm.tmp[w];
#pragma unroll
            for (int w = 0; w < kTileWaves; ++w) {
                sm.cnt[w][tid] = static_cast<uint16_t>(at);
                at += c[w];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTileRows; ++r) {
            if (!val[r]) continue;
            const uint32_t at = sm.cnt[wave][dig[r]] + before[r];
            if (at < kSortTile) {  // always, for a consistent count; keeps the stores inside
                sm.key[1 - src][at] = kv[r];
                sm.idx[1 - src][at] = iv[r];
            }
        }
        __syncthreads();
        src = 1 - src;
    }
    return src;
}

// ---- the whole cell table of a table of one tile ------------------------------------
// Tables of at most kSortTile particles and kTileCells cells are built by one
// workgroup (tile.hip): keys, tile_sort, the cell start/end table,
// cell_first and the reorder in one kernel.
constexpr uint32_t kTileCells = 8192;

inline bool one_tile_build(uint32_t n, uint32_t n_cells) { return n > 0 && n <= kSortTile && n_cells <= kTileCells; }

hipError_t launch_build_tile(const Plan& P, void* ws, StateDev in, StateDev sorted, const nauticle_cells& cells,
                             hipStream_t s);

hipError_t launch_radix_sort(uint32_t* const keys[2], uint32_t* const vals[2], uint32_t n, int bits,
                             bool ordered, uint32_t* hist, uint32_t* totals, hipStream_t s);

}  // namespace nau
