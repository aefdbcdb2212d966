// The whole cell table of a table of at most one sort tile (gfx950), built
// by one workgroup: keys, their stable sort in LDS (tile_sort), the cell
// start/end table, cell_first and the reorder in one kernel.
//
// Such tables are bound by latency.  The general path's dependent launches
// (two fills, keys, three kernels per sort pass, ranges, cell_first, reorder)
// each cost more than their work here.  The cell table comes from binary
// searches of the sorted keys in LDS, per cell: first[c] is the first
// position whose key is >= c, and a cell is occupied where first[c + 1] >
// first[c].  Each thread takes a run of consecutive cells, so the tables stay
// small (kTileCells).  The results are those of the general path, bit for
// bit.
#include "sort.h"

namespace nau {

__device__ inline uint32_t lower_bound_u32(const uint32_t* k, uint32_t lo, uint32_t hi, uint32_t c)
{
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (k[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Each phase issues all its global loads before it uses any: a thread's
// kTileIters particles (or items) are loaded together, and each particle's
// case comes from LDS (s_case), so every phase costs one trip to memory.
__global__ void __launch_bounds__(kTileThreads)
k_build_tile(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, uint32_t n,
             uint32_t n_cells, int bits, int dim_max, StateDev in, StateDev out, uint32_t* __restrict__ cell_key,
             uint32_t* __restrict__ perm, uint32_t* __restrict__ start, uint32_t* __restrict__ end,
             uint32_t* __restrict__ first, float4* __restrict__ pos4)
{
    __shared__ TileSort sm;
    __shared__ uint32_t s_case[kSortTile];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t wave = tid / kWave;
    // each particle's case: every item's first particle is marked with its
    // case + 1 and a prefix maximum carries the mark over the item (cases,
    // and so marks, grow with the particle index); n_items <= n <= kSortTile
    // = kTileIters threads' worth of items, so every item is loaded at once
    for (uint32_t i = tid; i < kSortTile; i += kTileThreads) s_case[i] = 0u;
    __syncthreads();
    {
        Item it[kTileIters];
#pragma unroll
        for (int k = 0; k < kTileIters; ++k) {
            const uint32_t ix = k * kTileThreads + tid;
            it[k] = items[ix < n_items ? ix : 0u];
            if (ix >= n_items) it[k].count = 0;
        }
#pragma unroll
        for (int k = 0; k < kTileIters; ++k)
            if (it[k].count > 0 && it[k].first < kSortTile) s_case[it[k].first] = it[k].case_id + 1u;
    }
    __syncthreads();
    {
        // thread t holds places 4t .. 4t + 3: a running maximum there, an
        // inclusive maximum over the wave's threads, then over the waves
        constexpr uint32_t kPer = kSortTile / kTileThreads;
        uint32_t v[kPer];
        uint32_t run = 0u;
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            run = max(run, s_case[tid * kPer + j]);
            v[j] = run;
        }
        uint32_t inc = run;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, kWave);
            if (lane >= static_cast<uint32_t>(d)) inc = max(inc, o);
        }
        __shared__ uint32_t s_wave_max[kTileWaves];
        if (lane == kWave - 1) s_wave_max[wave] = inc;
        __syncthreads();
        uint32_t before = __shfl_up(inc, 1, kWave);
        if (lane == 0) before = 0u;
        for (uint32_t w = 0; w < wave; ++w) before = max(before, s_wave_max[w]);
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) s_case[tid * kPer + j] = max(before, v[j]) - 1u;  // every place < n is marked
    }
    __syncthreads();
    {
        // loads at a valid position for every lane (n >= 1), used where live
        uint32_t cell[kTileIters], cid[kTileIters];
#pragma unroll
        for (int k = 0; k < kTileIters; ++k) {
            const uint32_t i = k * kTileThreads + tid;
            const uint32_t at = i < n ? i : 0u;
            cell[k] = in.cell[at];
            cid[k] = s_case[at];
        }
#pragma unroll
        for (int k = 0; k < kTileIters; ++k) {
            const uint32_t i = k * kTileThreads + tid;
            const CaseDev& C = cases[cid[k]];
            // a corrupt cell index: keep the key inside the case
            const uint32_t c = cell[k] < C.n_cells ? cell[k] : C.n_cells - 1;
            if (i < n) {
                sm.key[0][i] = C.cell_base + c;
                sm.idx[0][i] = static_cast<uint16_t>(i);
            }
        }
    }
    const int src = tile_sort(sm, n, bits);
    const uint32_t* key = sm.key[src];
    const uint16_t* idx = sm.idx[src];
    for (uint32_t i = tid; i < n; i += kTileThreads) {
        cell_key[i] = key[i];
        perm[i] = idx[i];
    }
    const uint32_t per = (n_cells + 1 + kTileThreads - 1) / kTileThreads;
    const uint32_t c_begin = tid * per;
    const uint32_t c_end = min(c_begin + per, n_cells + 1);
    if (c_begin < c_end) {
        uint32_t f = lower_bound_u32(key, 0, n, c_begin);
        for (uint32_t c = c_begin; c < c_end; ++c) {
            first[c] = f;
            if (c == n_cells) break;
            const uint32_t fn = lower_bound_u32(key, f, n, c + 1);
            const bool occupied = fn > f;
            start[c] = occupied ? f : NAUTICLE_EMPTY;
            end[c] = occupied ? fn : NAUTICLE_EMPTY;
            f = fn;
        }
    }
    // the reorder (as k_reorder): sorting keeps every particle inside its
    // case's range, so sorted position p has the case of input position p.
    // The state holds dim_max components for every particle; every load is
    // issued at a valid position (n >= 1) before any store.
    uint32_t q[kTileIters], cid[kTileIters], cell[kTileIters], id[kTileIters], ncx[kTileIters];
    int dim[kTileIters];
    float rho[kTileIters], o[kTileIters][3], v[kTileIters][3];
#pragma unroll
    for (int k = 0; k < kTileIters; ++k) {
        const uint32_t p = k * kTileThreads + tid;
        const uint32_t at = p < n ? p : 0u;
        q[k] = idx[at];
        cid[k] = s_case[at];
    }
#pragma unroll
    for (int k = 0; k < kTileIters; ++k) {
        const CaseDev& C = cases[cid[k]];
        ncx[k] = static_cast<uint32_t>(C.nc[0]);
        dim[k] = C.dim;
        cell[k] = in.cell[q[k]];
        id[k] = in.id[q[k]];
        rho[k] = 0.0f;
        if (in.rho) rho[k] = in.rho[q[k]];
        for (int a = 0; a < 3; ++a) {
            o[k][a] = 0.0f;
            v[k][a] = 0.0f;
            if (a < dim_max) {
                o[k][a] = in.off[a][q[k]];
                v[k][a] = in.vel[a][q[k]];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kTileIters; ++k) {
        const uint32_t p = k * kTileThreads + tid;
        if (p >= n) continue;
        out.cell[p] = cell[k];
        out.id[p] = id[k];
        if (in.rho) out.rho[p] = rho[k];
        for (int a = 0; a < 3; ++a) {
            if (a >= dim[k]) {
                o[k][a] = 0.0f;
                continue;
            }
            out.off[a][p] = o[k][a];
            out.vel[a][p] = v[k][a];
        }
        pos4[p] = make_float4(o[k][0], o[k][1], o[k][2], static_cast<float>(cell[k] % ncx[k]));
    }
}

hipError_t launch_build_tile(const Plan& P, void* ws, StateDev in, StateDev sorted, const nauticle_cells& cells,
                             hipStream_t s)
{
    const Packed pk = packed(P, ws);
    k_build_tile<<<1, kTileThreads, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items), P.n_items,
                                            P.n_total, P.n_cells_total, P.key_bits, P.dim_max, in, sorted, cells.key,
                                            cells.perm, cells.cell_start, cells.cell_end, pk.cell_first, pk.pos4);
    return hipGetLastError();
}

}  // namespace nau
