// Neighbour search on gfx950: binning, cell keys, their stable sort (in
// sort.hip), cell start/end table, reorder, and the per-particle neighbour
// lists.
//
// The cell grid follows the paper's domain (Sec. 3.2.1): cuboid cells no
// smaller than the influence radius, so every neighbour of a particle lies in
// the 3^dim block of cells around its own.  Keys are linear cell indices with
// x fastest, offset by the case's first key, so one global sort orders every
// case of a batch at once and a row of cells along x is contiguous in sorted
// order.
#include "sort.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace nau {

// ----------------------------------------------------------------------------
// binning: absolute FP32 positions -> (cell, offset), id
// ----------------------------------------------------------------------------

__global__ void __launch_bounds__(kMaxBlock)
k_bin(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items,
      const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz, StateDev st,
      uint32_t* err)
{
#pragma clang fp contract(off)
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const float* pos[3] = {px, py, pz};
    int32_t c[3] = {0, 0, 0};
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        if (k >= C.dim) break;
        float x = pos[k][i];
        if (!isfinite(x)) {
            set_error(err, kErrNonFinite);
            x = C.origin[k];
        }
        float t = x - C.origin[k];
        float r;
        ok &= split_offset(t, C.cs[k], C.inv_cs[k], C.nc[k], 0, &c[k], &r);
        st.off[k][i] = r;
    }
    if (!ok) set_error(err, kErrOutOfDomain);
    st.cell[i] = static_cast<uint32_t>(c[0]) +
                 static_cast<uint32_t>(C.nc[0]) * (static_cast<uint32_t>(c[1]) +
                                                   static_cast<uint32_t>(C.nc[1]) * static_cast<uint32_t>(c[2]));
    st.id[i] = i - C.offset;
}

__global__ void __launch_bounds__(kMaxBlock)
k_unbin(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
        float* px, float* py, float* pz, bool by_id)
{
#pragma clang fp contract(off)
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    uint32_t o = i;
    if (by_id) {
        uint32_t k = st.id[i];
        if (k >= C.n) k = C.n - 1;  // corrupt id: keep the write inside the case
        o = C.offset + k;
    }
    int32_t c[3];
    cell_coords(C, st.cell[i], c);
    float* pos[3] = {px, py, pz};
    for (int k = 0; k < 3; ++k) {
        if (k >= C.dim) break;
        float corner = C.origin[k] + static_cast<float>(c[k]) * C.cs[k];
        pos[k][o] = corner + st.off[k][i];
    }
}

// out[k][p] = g[k][offset + id[p]]: a per-particle vector given in input
// (id) order brought into the state's order.
__global__ void __launch_bounds__(kMaxBlock)
k_gather_id(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items,
            const uint32_t* __restrict__ id, const float* g0, const float* g1, const float* g2, float* o0,
            float* o1, float* o2)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t p = it.first + threadIdx.x;
    uint32_t k = id[p];
    if (k >= C.n) k = C.n - 1;
    const uint32_t q = C.offset + k;
    const float* g[3] = {g0, g1, g2};
    float* o[3] = {o0, o1, o2};
    for (int a = 0; a < 3; ++a) {
        if (a >= C.dim) break;
        o[a][p] = g[a][q];
    }
}

hipError_t launch_bin(const Plan& P, void* ws, const float* const pos[3], StateDev st, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    k_bin<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                 P.n_items, pos[0], pos[1], pos[2], st,
                                                 at<uint32_t>(ws, P.L.err));
    return hipGetLastError();
}

hipError_t launch_unbin(const Plan& P, void* ws, StateDev st, float* const pos[3], bool by_id, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    k_unbin<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                   P.n_items, st, pos[0], pos[1], pos[2], by_id);
    return hipGetLastError();
}

hipError_t launch_gather_id(const Plan& P, void* ws, const uint32_t* id, const float* const g[3],
                            float* const out[3], hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    k_gather_id<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                       P.n_items, id, g[0], g[1], g[2], out[0], out[1], out[2]);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// keys
// ----------------------------------------------------------------------------

__global__ void __launch_bounds__(kMaxBlock)
k_make_keys(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items,
            const uint32_t* __restrict__ cell, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const uint32_t i = it.first + threadIdx.x;
    uint32_t c = cell[i];
    const CaseDev& C = cases[it.case_id];
    // a corrupt cell index would index outside the cell table: clamp it
    if (c >= C.n_cells) c = C.n_cells - 1;
    keys[i] = C.cell_base + c;
    vals[i] = i;
}

// ----------------------------------------------------------------------------
// cell table, reorder
// ----------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* __restrict__ a, uint32_t n, uint32_t v)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// The same fill, four words per thread with 16-byte stores (a 16-byte aligned).
constexpr uint32_t kFillWords = 4;

__global__ void k_fill_u32x4(uint32_t* __restrict__ a, uint32_t n, uint32_t v)
{
    const uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) * kFillWords;
    if (i + kFillWords <= n) {
        *reinterpret_cast<uint4*>(a + i) = make_uint4(v, v, v, v);
    } else {
        for (uint32_t k = i; k < n; ++k) a[k] = v;
    }
}

// Fills a[0 .. n) with v on s: 16-byte stores where a is 16-byte aligned.
hipError_t fill_u32(uint32_t* a, uint32_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (reinterpret_cast<uintptr_t>(a) % 16u == 0) {
        const uint32_t threads = (n + kFillWords - 1) / kFillWords;
        k_fill_u32x4<<<(threads + kBlock - 1) / kBlock, kBlock, 0, s>>>(a, n, v);
    } else {
        k_fill_u32<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(a, n, v);
    }
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_cell_ranges(const uint32_t* __restrict__ keys, uint32_t n, uint32_t* __restrict__ start,
              uint32_t* __restrict__ end)
{
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) start[k] = p;
    if (p == n - 1 || keys[p + 1] != k) end[k] = p + 1;
}

// cell_first[c] = first sorted position whose key is >= c, for every key c in
// [0, n_cells].  Unlike cell_start it is defined for empty cells too, so
// [cell_first[a], cell_first[b + 1]) is the sorted range of the cells a..b.
// For a non-empty cell it is cell_start[c]; for an empty one, the start of
// the next non-empty cell (starts grow with the key), i.e. the minimum of
// cell_start over c' >= c, with the empty marker 0xFFFFFFFF above every
// start.  A workgroup takes kCellsPerGroup cells: a suffix minimum over its
// cells (per thread, then across the threads in LDS), and past its last cell
// the first position whose key is beyond it (one binary search), or n.
constexpr uint32_t kCellsPerThread = 4;
constexpr uint32_t kCellsPerGroup = kCellsPerThread * kBlock;

template <bool kVec>  // start is 16-byte aligned
__global__ void __launch_bounds__(kBlock)
k_cell_first(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ start, uint32_t n, uint32_t n_cells,
             uint32_t* __restrict__ first)
{
    __shared__ uint32_t s_min[kBlock];
    __shared__ uint32_t s_after;
    const uint32_t c0 = blockIdx.x * kCellsPerGroup;
    if (threadIdx.x == 0) {  // first position whose key is >= the cell after this group's
        const uint32_t c_next = c0 + kCellsPerGroup;
        uint32_t lo = 0, hi = n;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (keys[mid] < c_next) lo = mid + 1;
            else hi = mid;
        }
        s_after = lo;
    }
    const uint32_t cb = c0 + threadIdx.x * kCellsPerThread;
    uint32_t v[kCellsPerThread];
    if (kVec && cb + kCellsPerThread <= n_cells) {  // one 16-byte load
        const uint4 w = *reinterpret_cast<const uint4*>(start + cb);
        v[0] = w.x;
        v[1] = w.y;
        v[2] = w.z;
        v[3] = w.w;
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kCellsPerThread; ++i) {
            const uint32_t c = cb + i;
            v[i] = c < n_cells ? start[c] : (c == n_cells ? n : 0xFFFFFFFFu);
        }
    }
#pragma unroll
    for (int i = static_cast<int>(kCellsPerThread) - 2; i >= 0; --i) v[i] = min(v[i], v[i + 1]);
    // suffix minimum across the threads: s_min[t] = min over threads t' >= t
    s_min[threadIdx.x] = v[0];
    __syncthreads();
    for (uint32_t d = 1; d < kBlock; d <<= 1) {
        const uint32_t o = threadIdx.x + d < kBlock ? s_min[threadIdx.x + d] : 0xFFFFFFFFu;
        __syncthreads();
        s_min[threadIdx.x] = min(s_min[threadIdx.x], o);
        __syncthreads();
    }
    const uint32_t later = min(threadIdx.x + 1 < kBlock ? s_min[threadIdx.x + 1] : 0xFFFFFFFFu, s_after);
#pragma unroll
    for (uint32_t i = 0; i < kCellsPerThread; ++i) {
        const uint32_t c = cb + i;
        if (c <= n_cells) first[c] = min(v[i], later);
    }
}

// Gathers the state into sorted order and packs each particle's offsets into
// one float4 for the neighbour search and the density pass; w holds the x
// index of the particle's cell (exact in FP32), from which the search forms
// its cell frame shift.
// Two items per workgroup, one particle of each per thread: the reads of
// both permutation entries, and then all the gathers, are in flight
// together.  Each particle costs two dependent trips to memory, so twice the
// particles per thread keep twice the bytes in flight.
constexpr uint32_t kReorderItems = 2;

__global__ void __launch_bounds__(kMaxBlock)
k_reorder(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items,
          const uint32_t* __restrict__ perm, uint32_t n, StateDev in, StateDev out, float4* __restrict__ pos4)
{
    const uint32_t n_groups = (n_items + kReorderItems - 1) / kReorderItems;
    const uint32_t gx = xcd_item(n_groups);
    if (gx >= n_groups) return;
    bool live[kReorderItems];
    uint32_t p[kReorderItems], q[kReorderItems], ncx[kReorderItems];
    int dim[kReorderItems];
#pragma unroll
    for (uint32_t h = 0; h < kReorderItems; ++h) {
        const uint32_t ix = gx * kReorderItems + h;
        live[h] = false;
        p[h] = 0;
        ncx[h] = 1;
        dim[h] = 0;
        if (ix < n_items) {
            const Item it = items[ix];
            const CaseDev& C = cases[it.case_id];
            live[h] = threadIdx.x < it.count;
            p[h] = it.first + threadIdx.x;
            ncx[h] = static_cast<uint32_t>(C.nc[0]);
            dim[h] = C.dim;
        }
    }
#pragma unroll
    for (uint32_t h = 0; h < kReorderItems; ++h) {
        q[h] = live[h] ? perm[p[h]] : 0u;
        if (q[h] >= n) q[h] = p[h] < n ? p[h] : 0u;  // never for a permutation; guards memory
    }
    uint32_t cell[kReorderItems], id[kReorderItems];
    float rho[kReorderItems], o[kReorderItems][3], v[kReorderItems][3];
#pragma unroll
    for (uint32_t h = 0; h < kReorderItems; ++h) {
        if (!live[h]) continue;
        cell[h] = in.cell[q[h]];
        id[h] = in.id[q[h]];
        rho[h] = in.rho ? in.rho[q[h]] : 0.0f;
        for (int k = 0; k < 3; ++k) {
            o[h][k] = k < dim[h] ? in.off[k][q[h]] : 0.0f;
            v[h][k] = k < dim[h] ? in.vel[k][q[h]] : 0.0f;
        }
    }
#pragma unroll
    for (uint32_t h = 0; h < kReorderItems; ++h) {
        if (!live[h]) continue;
        out.cell[p[h]] = cell[h];
        out.id[p[h]] = id[h];
        if (in.rho) out.rho[p[h]] = rho[h];
        for (int k = 0; k < 3; ++k) {
            if (k >= dim[h]) break;
            out.off[k][p[h]] = o[h][k];
            out.vel[k][p[h]] = v[h][k];
        }
        pos4[p[h]] = make_float4(o[h][0], o[h][1], o[h][2], static_cast<float>(cell[h] % ncx[h]));
    }
}

__global__ void __launch_bounds__(kMaxBlock)
k_pack_positions(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items,
                 StateDev st, float4* __restrict__ pos4)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t p = it.first + threadIdx.x;
    float o[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < C.dim) o[k] = st.off[k][p];
    pos4[p] = make_float4(o[0], o[1], o[2], static_cast<float>(st.cell[p] % static_cast<uint32_t>(C.nc[0])));
}

hipError_t item_queue(const Plan& P, void* ws, int c, hipStream_t s, ItemQueue* Q)
{
    Q->n_items = P.n_items;
    Q->persistent = P.persistent;
    Q->order = at<uint32_t>(ws, P.L.queue);
    Q->counter = at<uint32_t>(ws, P.L.counters) + (c % kCounters) * kXcds * kCounterStride;
    if (!P.persistent) return hipSuccess;
    // a kernel, not a memset: safe under graph capture
    k_fill_u32<<<1, kXcds * kCounterStride, 0, s>>>(Q->counter, kXcds * kCounterStride, 0u);
    return hipGetLastError();
}

uint32_t persistent_groups(const Plan& P, const void* kernel, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<const void*, uint32_t, size_t>, int> fit;  // resident groups per CU
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        const auto key = std::make_tuple(kernel, P.block, lds);
        auto it = fit.find(key);
        if (it != fit.end()) {
            per_cu = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, static_cast<int>(P.block), lds) !=
                hipSuccess)
                per_cu = 1;
            fit.emplace(key, per_cu);
        }
    }
    if (per_cu < 1) per_cu = 1;
    const uint32_t g = P.groups_per_cu > 0 ? std::min<uint32_t>(P.groups_per_cu, per_cu) : per_cu;
    uint32_t groups = P.cus * g / kXcds * kXcds;
    groups = std::max<uint32_t>(groups, kXcds);
    return std::min(groups, xcd_grid(P.n_items));
}

hipError_t launch_cell_first(const Plan& P, void* ws, const nauticle_cells& cells, hipStream_t s)
{
    if (P.n_total == 0) return hipSuccess;
    const uint32_t nc = P.n_cells_total;
    auto cell_first = reinterpret_cast<uintptr_t>(cells.cell_start) % 16u == 0 ? k_cell_first<true>
                                                                               : k_cell_first<false>;
    cell_first<<<(nc + 1 + kCellsPerGroup - 1) / kCellsPerGroup, kBlock, 0, s>>>(cells.key, cells.cell_start,
                                                                                P.n_total, nc, packed(P, ws).cell_first);
    return hipGetLastError();
}

hipError_t launch_pack_positions(const Plan& P, void* ws, StateDev sorted, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    k_pack_positions<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                            P.n_items, sorted, packed(P, ws).pos4);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// neighbour lists
// ----------------------------------------------------------------------------
// One lane per sorted particle.  The 3^dim stencil is walked as 3^(dim-1)
// rows of three cells along x; since keys run x fastest, a row's three cells
// are one contiguous sorted range (two pieces where a periodic x axis wraps).
// The predicate subtracts the offsets first and adds the cell shift after,
// d = fl(fl(off_j - off_i) + delta cs), so the pair taken the other way round
// gives exactly -d and the relation is symmetric.  The y and z shifts are
// fixed per row; the x shift follows from the candidate's cell x index,
// packed with its offsets.
// Candidates come from the item's neighbourhood staged in LDS (global memory
// for folded pieces), kUnroll at a time with the next kUnroll in flight; those
// that pass set a bit in a 64-candidate mask, which is then emitted in
// ascending order into a four-entry register buffer that is stored as one
// 16-byte chunk when full.  Lanes of one home cell read the same candidate at
// the same time.  Reads may run up to 3 kUnroll - 1 candidates past a piece
// (LDS and the packed positions are padded for it); such candidates are
// masked off.

constexpr uint32_t kUnroll = 4;
static_assert(64 % (2 * kUnroll) == 0, "candidate groups must tile the 64-bit mask");
static_assert(3 * kUnroll <= kPosPad && 3 * kUnroll <= kHaloPad, "read-ahead past a piece must stay in the padding");

// The same test for a piece of mirror images: along an axis with sign -1
// the candidate's offset is negated, d = fl(fl(-off_j - off_i) + delta cs)
// (negation is exact), and a mirrored x piece (one boundary cell) takes
// cref = c_x - delta, delta 0 at the lower face and 2 at the upper one.
// With every sign +1 this is shift_group's arithmetic.
template <int DIM>
__device__ inline uint32_t test_group_img(const float4* o, float cref, float mex, float csx, float mey, float shy,
                                          float mez, float shz, float R2, float sx, float sy, float sz)
{
#pragma clang fp contract(off)
    uint32_t bits = 0;
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const float ddx = __builtin_fmaf(o[u].w - cref, csx, __builtin_fmaf(sx, o[u].x, -mex));
        const float ddy = __builtin_fmaf(sy, o[u].y, -mey) + shy;
        float r2 = __builtin_fmaf(ddy, ddy, ddx * ddx);
        if constexpr (DIM == 3) {
            const float ddz = __builtin_fmaf(sz, o[u].z, -mez) + shz;
            r2 = __builtin_fmaf(ddz, ddz, r2);
        }
        bits |= r2 < R2 ? (1u << u) : 0u;
    }
    return bits;
}

// Hit mask of the candidates q0 .. q0 + m - 1 (m <= 64) of a mirrored piece,
// read from `src` (a plain loop: such pieces are the few cells along a
// symmetric face).
template <int DIM>
__device__ inline uint64_t scan_chunk_img(const float4* src, uint32_t m, float cref, float mex, float csx, float mey,
                                          float shy, float mez, float shz, float R2, float sx, float sy, float sz)
{
    uint64_t hits = 0;
    for (uint32_t b = 0; b < m; b += kUnroll) {
        float4 o[kUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) o[u] = src[b + u];
        hits |= static_cast<uint64_t>(test_group_img<DIM>(o, cref, mex, csx, mey, shy, mez, shz, R2, sx, sy, sz))
                << b;
    }
    return hits;
}

// The distance test of one candidate group, shifted into a running mask:
// each candidate's bit enters at bit 0 and the earlier ones move up, so
// after n candidates candidate k sits at bit n - 1 - k.  The bit is the
// sign of fl(r2 - R2), which is r2 < R2 exactly: both are finite and
// non-negative, near R2 the difference is exact, elsewhere it is far from
// zero.  One subtraction and one funnel shift per candidate, instead of a
// compare, a select and the merging of group masks.  The candidate's cell x
// index (o.w) against the piece's reference gives delta_x in {-1, 0, 1}, so
// d_x = fl(fl(off_j - off_i) + delta_x cs) is one fused multiply-add of an
// exact product; the y and z shifts (shy, shz) are exact multiples of the
// cell edge, fixed per row.
template <int DIM>
__device__ inline uint32_t shift_group(const float4* o, float cref, float mex, float csx, float mey, float shy,
                                       float mez, float shz, float R2, uint32_t acc)
{
#pragma clang fp contract(off)
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const float ddx = __builtin_fmaf(o[u].w - cref, csx, o[u].x - mex);
        const float ddy = (o[u].y - mey) + shy;
        float r2 = __builtin_fmaf(ddy, ddy, ddx * ddx);
        if constexpr (DIM == 3) {
            const float ddz = (o[u].z - mez) + shz;
            r2 = __builtin_fmaf(ddz, ddz, r2);
        }
        acc = __builtin_amdgcn_alignbit(acc, __builtin_bit_cast(uint32_t, r2 - R2), 31u);
    }
    return acc;
}

// Hit mask (bit k = candidate k) of the candidates src[0 .. m-1], 1 <= m <=
// 32 (readable up to 3 kUnroll - 1 past m - 1).  Two groups per iteration in
// ping-pong registers: group A is tested while group B loads, then B while
// the next A loads (on the last pass a group past the end, read and not
// used, so the address needs no select).  The loop tests b = 8 ceil(m/8)
// candidates; the shifted mask is reversed and aligned at the end.
template <int DIM>
__device__ inline uint32_t scan32(const float4* src, uint32_t m, float cref, float mex, float csx, float mey,
                                  float shy, float mez, float shz, float R2)
{
    uint32_t acc = 0;
    float4 oa[kUnroll], ob[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) oa[u] = src[u];
    uint32_t b = 0;
    for (; b < m; b += 2 * kUnroll) {
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) ob[u] = src[b + kUnroll + u];
        __builtin_amdgcn_sched_barrier(0);
        acc = shift_group<DIM>(oa, cref, mex, csx, mey, shy, mez, shz, R2, acc);
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) oa[u] = src[b + 2 * kUnroll + u];
        __builtin_amdgcn_sched_barrier(0);
        acc = shift_group<DIM>(ob, cref, mex, csx, mey, shy, mez, shz, R2, acc);
    }
    return __builtin_bitreverse32(acc) >> (32u - b);  // 8 <= b <= 32
}

// Hit mask of the candidates q0 .. q0 + m - 1 (m <= 64) read from `src`
// (src[k] = candidate q0 + k; readable up to 3 kUnroll - 1 past m - 1), as
// two halves of 32.
template <int DIM>
__device__ inline uint64_t scan_chunk(const float4* src, uint32_t m, float cref, float mex, float csx, float mey,
                                      float shy, float mez, float shz, float R2)
{
    const uint32_t lo = scan32<DIM>(src, m < 32u ? m : 32u, cref, mex, csx, mey, shy, mez, shz, R2);
    const uint32_t hi = m > 32u ? scan32<DIM>(src + 32, m - 32u, cref, mex, csx, mey, shy, mez, shz, R2) : 0u;
    return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
}

// Appends the entries of the hits (ascending) to a lane's list: each enters
// a four-entry register buffer (newest in w), stored as one 16-byte chunk
// when full.  The entry of candidate q0 + b is e0 + b plus one x step of the
// offset code per cell boundary (r1, r2, relative to q0) at or before b; the
// three bases are formed once.  kCheck: stop storing past max_nbr entries
// (the count still grows).
template <bool kCheck>
__device__ inline void emit_hits(uint64_t hits, uint32_t e0, int32_t r1, int32_t r2, uint4& buf, uint32_t& cnt,
                                 uint4*& dst, uint32_t n_total, uint32_t max_nbr)
{
    constexpr uint32_t kStep = 1u << NAUTICLE_NBR_INDEX_BITS;
    const uint32_t e1 = e0 + kStep, e2 = e0 + 2u * kStep;
    while (hits) {
        const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(hits));
        hits &= hits - 1;
        const int32_t sb = static_cast<int32_t>(b);
        const uint32_t base = sb >= r2 ? e2 : (sb >= r1 ? e1 : e0);
        buf.x = buf.y;
        buf.y = buf.z;
        buf.z = buf.w;
        buf.w = base + b;
        ++cnt;
        if ((cnt & 3u) == 0u && (!kCheck || cnt <= max_nbr)) {
            *dst = buf;
            dst += n_total;
        }
    }
}

// kMirror: the case may have symmetric faces.  A stencil cell beyond such a
// face stands for the mirror image of the particle's own boundary cell: its
// rows (y, z) or its piece (x) are the boundary cell's particles with the
// offsets along that axis negated, entered with offset code kMirrorCode; the
// particle's own image is a neighbour like any other.
template <int DIM, bool kMirror>
__device__ inline void nlist_particle(const CaseDev& C, const Item& it, StateDev st, const float4* __restrict__ pos4,
                                      const HaloRows& H, const float4* halo,
                                      const uint32_t* __restrict__ cell_first, uint32_t* __restrict__ nbr,
                                      uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total,
                                      uint32_t* err)
{
#pragma clang fp contract(off)
    const uint32_t p = it.first + threadIdx.x;
    uint32_t own = st.cell[p];
    if (own >= C.n_cells) {  // a corrupt state: keep every table access inside the case
        own = C.n_cells - 1;
        set_error(err, kErrOutOfDomain);
    }
    int32_t c[3];
    cell_coords(C, own, c);
    const float4 me = pos4[p];
    const float R2 = C.R2;
    const int32_t nx = C.nc[0];
    const bool px = C.periodic[0] != 0;
    const float csx = C.cs[0];
    uint4* col = reinterpret_cast<uint4*>(nbr) + p;  // chunk c at col[c * n_total]
    const uint32_t max_chunks = max_nbr / kChunk;
    uint4* dst = col;  // where the next full chunk goes (advanced by n_total chunks)
    uint4 buf = make_uint4(0u, 0u, 0u, 0u);  // the last four entries, newest in w
    uint32_t cnt = 0;
    constexpr int kZ = DIM == 3 ? 1 : 0;
    for (int dz = -kZ; dz <= kZ; ++dz) {
        int32_t cz = c[2] + dz;
        bool mz = false;  // this plane is the mirror image of the particle's own
        if constexpr (DIM == 3) {
            if (C.periodic[2]) {
                cz = cz < 0 ? cz + C.nc[2] : (cz >= C.nc[2] ? cz - C.nc[2] : cz);
            } else if (cz < 0 || cz >= C.nc[2]) {
                if (!kMirror || !C.mirror[2]) continue;
                cz = c[2];
                mz = true;
            }
        }
        // the cell shift: delta cells, or 0 / 2 cells against a lower /
        // upper face for an image plane (an exact multiple of the edge)
        const float shz = static_cast<float>(mz ? (dz < 0 ? 0 : 2) : dz) * C.cs[2];
        for (int dy = -1; dy <= 1; ++dy) {
            int32_t cy = c[1] + dy;
            bool my = false;
            if (C.periodic[1]) {
                cy = cy < 0 ? cy + C.nc[1] : (cy >= C.nc[1] ? cy - C.nc[1] : cy);
            } else if (cy < 0 || cy >= C.nc[1]) {
                if (!kMirror || !C.mirror[1]) continue;
                cy = c[1];
                my = true;
            }
            const uint32_t row = C.cell_base + static_cast<uint32_t>(nx) *
                                                   (static_cast<uint32_t>(cy) + static_cast<uint32_t>(C.nc[1]) * static_cast<uint32_t>(cz));
            const float shy = static_cast<float>(my ? (dy < 0 ? 0 : 2) : dy) * C.cs[1];
            // the row's x span [c-1, c+1] as up to two contiguous pieces of
            // cells; the second is the wrapped cell of a periodic x axis or
            // the image of the boundary cell of a symmetric one
            int32_t lo0 = c[0] - 1, hi0 = c[0] + 1, lo1 = 0, hi1 = -1;
            bool mx1 = false;    // piece 1 is an image piece
            int32_t dimg = 0;    // its shift in cells: 0 (lower face) or 2 (upper)
            if (px) {
                if (lo0 < 0) { lo1 = nx - 1; hi1 = nx - 1; lo0 = 0; }
                if (hi0 >= nx) { lo1 = 0; hi1 = 0; hi0 = nx - 1; }
            } else {
                const bool img = kMirror && C.mirror[0];
                if (lo0 < 0) {
                    lo0 = 0;
                    if (img) { lo1 = 0; hi1 = 0; mx1 = true; dimg = 0; }
                }
                if (hi0 >= nx) {
                    hi0 = nx - 1;
                    if (img) { lo1 = nx - 1; hi1 = nx - 1; mx1 = true; dimg = 2; }
                }
            }
            const uint32_t code_yz = ((my ? kMirrorCode : static_cast<uint32_t>(dy + 1)) << (NAUTICLE_NBR_INDEX_BITS + 2)) |
                                     ((mz ? kMirrorCode : static_cast<uint32_t>(dz + 1)) << (NAUTICLE_NBR_INDEX_BITS + 4));
            for (int piece = 0; piece < 2; ++piece) {
                const int32_t xa = piece == 0 ? lo0 : lo1;
                const int32_t xb = piece == 0 ? hi0 : hi1;
                if (xb < xa) continue;
                const bool mx = piece == 1 && mx1;
                const uint32_t q_begin = min(cell_first[row + static_cast<uint32_t>(xa)], n_total);
                const uint32_t q_end = min(cell_first[row + static_cast<uint32_t>(xb) + 1], n_total);
                // cell x offset of the piece's first cell, where its next cells
                // start, and the particle's x in each of those cells' frames
                // (an image piece is one cell: code kMirrorCode = dx0 + 1)
                int32_t dx0 = xa - c[0];
                if (mx) dx0 = static_cast<int32_t>(kMirrorCode) - 1;
                else if (dx0 > 1) dx0 -= nx;
                else if (dx0 < -1) dx0 += nx;
                const uint32_t b1 = xa + 1 <= xb ? cell_first[row + static_cast<uint32_t>(xa) + 1] : q_end;
                const uint32_t b2 = xa + 2 <= xb ? cell_first[row + static_cast<uint32_t>(xa) + 2] : q_end;
                // candidate cell x index - cref = delta_x (the wrapped piece's
                // single cell included); for an image piece, -(its shift)
                const float cref = static_cast<float>(mx ? c[0] - dimg : xa - dx0);
                const bool image = mx || my || mz;
                // the piece from LDS when it lies in the staged range of the
                // row that holds its cells
                const uint32_t hr = halo_row<DIM>(my ? 0 : dy, mz ? 0 : dz);
                const bool staged = q_begin >= H.lo[hr] && q_end <= H.hi[hr];
                const int32_t hshift = H.shift[hr];
                for (uint32_t q0 = q_begin; q0 < q_end; q0 += 64) {
                    const uint32_t m = min(q_end - q0, 64u);
                    const float4* src = staged ? halo + (static_cast<int32_t>(q0) + hshift) : pos4 + q0;
                    uint64_t hits_all;
                    if (kMirror && image)
                        hits_all = scan_chunk_img<DIM>(src, m, cref, me.x, csx, me.y, shy, me.z, shz, R2,
                                                       mx ? -1.0f : 1.0f, my ? -1.0f : 1.0f, mz ? -1.0f : 1.0f);
                    else
                        hits_all = staged ? scan_chunk<DIM>(halo + (static_cast<int32_t>(q0) + hshift), m, cref, me.x,
                                                            csx, me.y, shy, me.z, shz, R2)
                                          : scan_chunk<DIM>(pos4 + q0, m, cref, me.x, csx, me.y, shy, me.z, shz, R2);
                    uint64_t hits = hits_all;
                    // drop candidates past the piece and the particle itself
                    // (its own image stays)
                    if (m < 64) hits &= (uint64_t{1} << m) - 1u;
                    if (p - q0 < 64u && !(kMirror && image)) hits &= ~(uint64_t{1} << (p - q0));
                    // entry of candidate q0 + b: the index plus the piece's first-cell
                    // code (the fields do not overlap), plus one x step per cell
                    // boundary at or before it
                    const uint32_t e0 =
                        q0 + (code_yz | (static_cast<uint32_t>(dx0 + 1) << NAUTICLE_NBR_INDEX_BITS));
                    // boundaries relative to q0 (negative if before it)
                    const int32_t r1 = static_cast<int32_t>(b1 - q0), r2 = static_cast<int32_t>(b2 - q0);
                    // a list with room for every hit of the chunk stores them
                    // without the capacity test
                    if (cnt + static_cast<uint32_t>(__popcll(hits)) <= max_nbr)
                        emit_hits<false>(hits, e0, r1, r2, buf, cnt, dst, n_total, max_nbr);
                    else
                        emit_hits<true>(hits, e0, r1, r2, buf, cnt, dst, n_total, max_nbr);
                }
            }
        }
    }
    // the last, partial chunk: its r entries are the newest r of the buffer,
    // the rest padding
    const uint32_t r = cnt & 3u;
    if (r != 0u && (cnt >> 2) < max_chunks) {
        const uint32_t z = pad_entry(p, DIM);
        const uint4 out = r == 1u ? make_uint4(buf.w, z, z, z)
                                  : (r == 2u ? make_uint4(buf.z, buf.w, z, z) : make_uint4(buf.y, buf.z, buf.w, z));
        col[static_cast<size_t>(cnt >> 2) * n_total] = out;
    }
    nbr_count[p] = cnt;
    if (cnt > max_nbr) set_error(err, kErrOverflow);
}

// The search is bound by the latency of each wave's dependent LDS reads and
// emission steps, so it runs as many items per CU as fit: the LDS halo
// (kHaloBytes) admits five of 256 particles, and five waves per SIMD hold
// the kernel to 96 VGPRs (no spill without symmetric faces; 8 registers
// spilled with them).
template <int DIM, bool kMirror>
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(5)))
k_nlist(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
        const float4* __restrict__ pos4, const uint32_t* __restrict__ cell_first, uint32_t* __restrict__ nbr,
        uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total, uint32_t halo_cap, uint32_t* err)
{
    extern __shared__ float4 s_halo[];  // halo_cap + kHaloPad records
    __shared__ HaloRows s_rows;
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        halo_plan<DIM>(C, it, st.cell, cell_first, n_total, halo_cap, &s_rows);
        halo_copy<DIM>(s_rows, pos4, s_halo);
        if (threadIdx.x < it.count)
            nlist_particle<DIM, kMirror>(C, it, st, pos4, s_rows, s_halo, cell_first, nbr, nbr_count, max_nbr,
                                         n_total, err);
        __syncthreads();  // the next item's staging overwrites the LDS
    });
}

// ----------------------------------------------------------------------------
// build_cells
// ----------------------------------------------------------------------------

// The general path: keys, the radix sort, the cell ranges over filled
// tables, cell_first and the reorder, each its own launch.
static hipError_t build_table(const Plan& P, void* ws, StateDev in, StateDev sorted, const nauticle_cells& cells,
                              hipStream_t s)
{
    const uint32_t n = P.n_total;
    const uint32_t nc = P.n_cells_total;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    const Packed pk = packed(P, ws);
    if (nc > 0) {
        hipError_t fe = fill_u32(cells.cell_start, nc, NAUTICLE_EMPTY, s);
        if (fe == hipSuccess) fe = fill_u32(cells.cell_end, nc, NAUTICLE_EMPTY, s);
        if (fe != hipSuccess) return fe;
    }
    if (n == 0) return hipGetLastError();

    // stable radix sort of (key, index); started in the buffer pair that makes
    // the last pass land in cells.key / cells.perm
    uint32_t* const ws_keys = at<uint32_t>(ws, P.L.sort_keys);
    uint32_t* const ws_vals = at<uint32_t>(ws, P.L.sort_vals);
    const bool even = radix_passes(P.key_bits) % 2 == 0;
    uint32_t* const keys[2] = {even ? cells.key : ws_keys, even ? ws_keys : cells.key};
    uint32_t* const vals[2] = {even ? cells.perm : ws_vals, even ? ws_vals : cells.perm};
    k_make_keys<<<xcd_grid(P.n_items), P.block, 0, s>>>(cases, items, P.n_items, in.cell, keys[0], vals[0]);
    // fewer particles than cells: consecutive keys mostly differ, and the
    // sort's scatter orders each tile in LDS before storing it
    const bool sparse = n < nc;
    hipError_t e = launch_radix_sort(keys, vals, n, P.key_bits, sparse, at<uint32_t>(ws, P.L.sort_hist),
                                     at<uint32_t>(ws, P.L.sort_totals), s);
    if (e != hipSuccess) return e;
    const int nb = static_cast<int>((n + kBlock - 1) / kBlock);
    k_cell_ranges<<<nb, kBlock, 0, s>>>(cells.key, n, cells.cell_start, cells.cell_end);
    auto cell_first = reinterpret_cast<uintptr_t>(cells.cell_start) % 16u == 0 ? k_cell_first<true>
                                                                               : k_cell_first<false>;
    cell_first<<<(nc + 1 + kCellsPerGroup - 1) / kCellsPerGroup, kBlock, 0, s>>>(cells.key, cells.cell_start, n, nc,
                                                                                pk.cell_first);
    const uint32_t reorder_groups = (P.n_items + kReorderItems - 1) / kReorderItems;
    k_reorder<<<xcd_grid(reorder_groups), P.block, 0, s>>>(cases, items, P.n_items, cells.perm, n, in, sorted, pk.pos4);
    return hipGetLastError();
}

hipError_t launch_build_cells(const Plan& P, void* ws, StateDev in, StateDev sorted,
                              const nauticle_cells& cells, hipStream_t s, hipEvent_t mid)
{
    const uint32_t n = P.n_total;
    const uint32_t nc = P.n_cells_total;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    uint32_t* err = at<uint32_t>(ws, P.L.err);
    const Packed pk = packed(P, ws);
    if (one_tile_build(n, nc)) {
        const hipError_t e = launch_build_tile(P, ws, in, sorted, cells, s);
        if (e != hipSuccess) return e;
    } else {
        const hipError_t e = build_table(P, ws, in, sorted, cells, s);
        if (e != hipSuccess || n == 0) return e;
    }
    ItemQueue Q;
    hipError_t e = item_queue(P, ws, 0, s, &Q);
    if (e == hipSuccess && mid) e = hipEventRecord(mid, s);
    if (e != hipSuccess) return e;
    const uint32_t mx = static_cast<uint32_t>(cells.max_nbr);
    const uint32_t cap = halo_records(P.halo_cap, 1, kHaloBytes);
    const size_t lds = sizeof(float4) * (cap + kHaloPad);
    auto kern = P.dim_max == 3 ? (P.mirror ? k_nlist<3, true> : k_nlist<3, false>)
                               : (P.mirror ? k_nlist<2, true> : k_nlist<2, false>);
    kern<<<grid_for(P, reinterpret_cast<const void*>(kern), lds), P.block, lds, s>>>(
        cases, items, Q, sorted, pk.pos4, pk.cell_first, cells.nbr, cells.nbr_count, mx, n, cap, err);
    return hipGetLastError();
}

}  // namespace nau
