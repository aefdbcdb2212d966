// Stable LSD radix sort of (key, value) pairs on gfx950.
//
// Per pass (a digit of at most 8 bits at `shift`):
//   1. k_rs_hist:    per tile of kSortTile keys, digit histogram -> hist[d][tile]
//   2. k_rs_scan:    per digit, exclusive scan over the tiles; digit totals
//   3. k_rs_scatter: per tile, each key's rank among the tile's keys of its
//                    digit, in input order (wave ballots for the lanes of a
//                    wave, LDS counters across waves and iterations), and the
//                    stable scatter; for sparse tables the tile is ordered by
//                    digit in LDS first, so that a wave stores to a few runs.
#include "sort.h"

namespace nau {

namespace {

constexpr int kItems = static_cast<int>(kSortTile) / kBlock;  // keys per thread per tile
static_assert(kItems * kBlock == static_cast<int>(kSortTile), "a tile is a whole number of block rows");
static_assert(kSortBins == static_cast<uint32_t>(kBlock), "one thread per digit");

// Inclusive scan across a wave64 with shuffles.
__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(v, d, kWave);
        if (lane >= static_cast<uint32_t>(d)) v += o;
    }
    return v;
}

// Exclusive scan over the 256 threads of a block; returns the block total in
// *total.  `tmp` must hold kBlock / kWave words.  Contains barriers; `tmp` is
// free again on return.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total)
{
    const uint32_t lane = __lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) tmp[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        uint32_t t = tmp[w];
        if (static_cast<uint32_t>(w) < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

}  // namespace

__global__ void __launch_bounds__(kBlock)
k_rs_hist(const uint32_t* __restrict__ keys, uint32_t n, int shift, uint32_t mask,
          uint32_t* __restrict__ hist, uint32_t n_tiles)
{
    __shared__ uint32_t h[kSortBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        uint32_t idx = base + k * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock)
k_rs_scan(uint32_t* __restrict__ hist, uint32_t n_tiles, uint32_t* __restrict__ totals)
{
    __shared__ uint32_t tmp[kBlock / kWave];
    uint32_t* row = hist + static_cast<size_t>(blockIdx.x) * n_tiles;
    uint32_t running = 0;
    constexpr int kPer = 4;
    for (uint32_t base = 0; base < n_tiles; base += kBlock * kPer) {
        uint32_t v[kPer];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            uint32_t idx = base + threadIdx.x * kPer + k;
            v[k] = idx < n_tiles ? row[idx] : 0u;
            sum += v[k];
        }
        uint32_t total;
        uint32_t ex = block_exclusive_scan(sum, tmp, &total);
        uint32_t acc = running + ex;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            uint32_t idx = base + threadIdx.x * kPer + k;
            if (idx < n_tiles) row[idx] = acc;
            acc += v[k];
        }
        running += total;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = running;
}

// hist[d][tile] holds, after k_rs_scan, the number of digit-d keys in the
// tiles before `tile`; totals[d] the number in all tiles.
//
// kOrdered: the tile is ordered by digit in LDS first and written out in that
// order, so the lanes of a wave store to a few runs.  Without it each key is
// stored at its place directly, which coalesces as well when consecutive keys
// share their digit (tables with several particles per cell), and then the
// LDS round trip and the occupancy it costs are a loss.
template <bool kOrdered>
__global__ void __launch_bounds__(kBlock)
k_rs_scatter(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t n,
             int shift, uint32_t mask, int bits, const uint32_t* __restrict__ hist,
             const uint32_t* __restrict__ totals, uint32_t n_tiles, uint32_t* __restrict__ keys_out,
             uint32_t* __restrict__ vals_out)
{
    // the staging arrays are used by the ordered variant only
    constexpr uint32_t kStage = kOrdered ? kSortTile : 1u;
    constexpr uint32_t kStageBins = kOrdered ? kSortBins : 1u;
    __shared__ uint32_t s_key[kStage];  // the tile ordered by digit, stably
    __shared__ uint32_t s_val[kStage];
    __shared__ uint32_t out_base[kStageBins];    // where the tile's digit-d keys go in the output
    __shared__ uint32_t tile_start[kStageBins];  // where they start in the tile's order
    __shared__ uint32_t next[kSortBins];        // the next free place of digit d (tile order, or output)
    __shared__ uint32_t wave_cnt[kBlock / kWave][kSortBins];
    __shared__ uint32_t tmp[kBlock / kWave];
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t wave = tid / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));

    // digit `tid`: its keys before this tile, and in it
    const uint32_t before = hist[static_cast<size_t>(tid) * n_tiles + tile];
    uint32_t total;
    const uint32_t base_out = block_exclusive_scan(totals[tid], tmp, &total) + before;
    if constexpr (kOrdered) {
        const uint32_t upto = tile + 1 < n_tiles ? hist[static_cast<size_t>(tid) * n_tiles + tile + 1] : totals[tid];
        const uint32_t start = block_exclusive_scan(upto - before, tmp, &total);
        out_base[tid] = base_out;
        tile_start[tid] = start;
        next[tid] = start;
    } else {
        next[tid] = base_out;
    }
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) wave_cnt[w][tid] = 0;
    __syncthreads();

    // the tile's keys and values, all loads in flight at once (the ranking
    // loop below has barriers, across which loads would not be moved)
    const uint32_t base = tile * kSortTile;
    uint32_t keys[kItems], vals[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t idx = base + k * kBlock + tid;
        keys[k] = idx < n ? keys_in[idx] : 0u;
        vals[k] = idx < n ? vals_in[idx] : 0u;
    }

    // each key's place among the tile's keys of its digit, in input order
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t idx = base + k * kBlock + tid;
        const bool valid = idx < n;
        const uint32_t key = keys[k];
        const uint32_t val = vals[k];
        const uint32_t d = (key >> shift) & mask;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wave_cnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t at = next[d] + rank;
            for (uint32_t w = 0; w < wave; ++w) at += wave_cnt[w][d];
            // the guards always hold for a consistent histogram; they keep
            // the stores inside LDS and the output
            if constexpr (kOrdered) {
                if (at < kStage) {
                    s_key[at] = key;
                    s_val[at] = val;
                }
            } else {
                if (at < n) {
                    keys_out[at] = key;
                    vals_out[at] = val;
                }
            }
        }
        __syncthreads();
        // advance each digit past this iteration's keys
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) {
            add += wave_cnt[w][tid];
            wave_cnt[w][tid] = 0;
        }
        next[tid] += add;
        __syncthreads();
    }

    if constexpr (kOrdered) {  // the tile in digit order to the output: a digit's keys are one run
        const uint32_t count = n - base < kSortTile ? n - base : kSortTile;
#pragma unroll 4
        for (int k = 0; k < kItems; ++k) {
            const uint32_t t = k * kBlock + tid;
            if (t < count) {
                const uint32_t key = s_key[t];
                const uint32_t d = (key >> shift) & mask;
                const uint32_t pos = out_base[d] + (t - tile_start[d]);
                if (pos < n) {
                    keys_out[pos] = key;
                    vals_out[pos] = s_val[t];
                }
            }
        }
    }
}

// A table of at most one tile: one workgroup sorts it in LDS (tile_sort in
// sort.h) and gathers the values once at the end.  The output buffers may be
// the input ones.  Separate launches of the three pass kernels would each
// cost a launch and leave all but one CU idle.
__global__ void __launch_bounds__(kTileThreads)
k_rs_tile(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t n, int bits, uint32_t* keys_out,
          uint32_t* vals_out)
{
    __shared__ TileSort sm;
    for (uint32_t i = threadIdx.x; i < n; i += kTileThreads) {
        sm.key[0][i] = keys_in[i];
        sm.idx[0][i] = static_cast<uint16_t>(i);
    }
    const int src = tile_sort(sm, n, bits);
    // the output may be the input (an even number of passes): every value
    // is read before any is stored
    uint32_t v[kTileIters];
#pragma unroll
    for (int k = 0; k < kTileIters; ++k) {
        const uint32_t i = k * kTileThreads + threadIdx.x;
        const uint32_t from = i < n ? sm.idx[src][i] : 0u;
        v[k] = i < n ? vals_in[from < n ? from : 0u] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTileIters; ++k) {
        const uint32_t i = k * kTileThreads + threadIdx.x;
        if (i < n) {
            keys_out[i] = sm.key[src][i];
            vals_out[i] = v[k];
        }
    }
}

hipError_t launch_radix_sort(uint32_t* const keys[2], uint32_t* const vals[2], uint32_t n, int bits,
                             bool ordered, uint32_t* hist, uint32_t* totals, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int passes = radix_passes(bits);
    if (n <= kSortTile) {  // the result lands where the pass-by-pass sort would leave it
        const int res = passes % 2;
        k_rs_tile<<<1, kTileThreads, 0, s>>>(keys[0], vals[0], n, bits, keys[res], vals[res]);
        return hipGetLastError();
    }
    const int per = (bits + passes - 1) / passes;
    const uint32_t n_tiles = (n + kSortTile - 1) / kSortTile;
    int src = 0;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * per;
        const int b = (bits - shift) < per ? (bits - shift) : per;
        const uint32_t mask = (1u << b) - 1u;
        k_rs_hist<<<n_tiles, kBlock, 0, s>>>(keys[src], n, shift, mask, hist, n_tiles);
        k_rs_scan<<<kSortBins, kBlock, 0, s>>>(hist, n_tiles, totals);
        auto scatter = ordered ? k_rs_scatter<true> : k_rs_scatter<false>;
        scatter<<<n_tiles, kBlock, 0, s>>>(keys[src], vals[src], n, shift, mask, b, hist, totals, n_tiles,
                                           keys[1 - src], vals[1 - src]);
        src = 1 - src;
    }
    return hipGetLastError();
}

}  // namespace nau
