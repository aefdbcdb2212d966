// Internal declarations of libnauticle (HIP, gfx950).  Not installed; the
// public interface is include/nauticle.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "nauticle.h"

namespace nau {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr uint32_t kPosPad = 64;   // float4s readable past the end of the packed position array
constexpr uint32_t kIndexMask = (1u << NAUTICLE_NBR_INDEX_BITS) - 1u;
constexpr int32_t kChunk = 4;      // list entries per 16-byte chunk

// The entry that fills a particle's list from its count to the end of the
// last chunk: the particle itself, one cell away along every axis of the
// case (offset code (-1, -1, -1), or (-1, -1, 0) in 2-D).  Its distance is
// at least sqrt(2) cell sizes > 2h, so every kernel term of such a pair is
// exactly zero and the pair loops need no per-pair mask.
__device__ inline uint32_t pad_entry(uint32_t p, int dim)
{
    return p | (dim == 3 ? 0u : (1u << (NAUTICLE_NBR_INDEX_BITS + 4)));
}

// Chunk c (entries 4c .. 4c + 3) of sorted particle p's neighbour list.
__device__ inline const uint4* nbr_chunk(const uint32_t* nbr, uint32_t c, uint32_t p, uint32_t n_total)
{
    return reinterpret_cast<const uint4*>(nbr) + (static_cast<size_t>(c) * n_total + p);
}

// Device error word bits (OR-ed by kernels, read by nauticle_check).
constexpr uint32_t kErrNonFinite = 1u;
constexpr uint32_t kErrOverflow = 2u;
constexpr uint32_t kErrOutOfDomain = 4u;
constexpr uint32_t kErrAttribute = 8u;

// Per-case constants, derived once on the host in FP64 and rounded to FP32.
struct CaseDev {
    int32_t dim;
    int32_t nc[3];
    int32_t periodic[3];
    int32_t mirror[3];   // symmetric faces (a cell beyond one stands for the boundary cell's image)
    uint32_t cell_base;  // first global cell key of the case
    uint32_t n_cells;
    uint32_t offset;     // first global particle
    uint32_t n;          // particles
    uint32_t n_fluid;    // ids >= n_fluid are fixed
    uint32_t item_first; // this case's blocks of particles in the item list
    uint32_t item_count;
    float cs[3];         // fl32(cell_size)
    float inv_cs[3];     // fl32(1 / cell_size)
    float origin[3];     // fl32(origin)
    float R2;            // fl32((2h + skin)^2): the neighbour lists' reach
    float inv_h;
    float m;             // particle mass
    float m_alpha;       // m * alpha_D (self density, and W's scale)
    float F_coef;        // -5 alpha_D / h^2   (F = F_coef (1 - q/2)^3)
    float dF_coef;       // 15 alpha_D / (2 h^3)  (F' = dF_coef (1 - q/2)^2)
    float rho0, inv_rho0, B, gamma, c0;
    float nu, dt;
    float g[3];
    float c2;            // c0^2 (linear equation of state)
    float av_coef;       // alpha_av c0 h m (artificial viscosity, times 1/rho_i per particle)
    float h;             // smoothing length (pair laws: the largest radius allowed)
    float law[4];        // pair-law constants (DEM: c_f; social force: A, B, k, tau)
    float verlet_lim2;   // fl32(lim^2): a displacement beyond lim since the last build forces one
};

// Offset code of a list entry along axis k (bits 26 + 2k, 27 + 2k): the
// neighbour's cell minus the particle's cell plus one, or kMirrorCode for the
// mirror image of a neighbour in a symmetric face of the particle's own
// (boundary) cell.
constexpr uint32_t kMirrorCode = 3u;

// A tile of at most kBlock consecutive particles of one case.
struct Item {
    uint32_t case_id;
    uint32_t first;
    uint32_t count;
    uint32_t pad;
};

// Device pointers of a state in the cell-relative layout.
struct StateDev {
    uint32_t* cell;
    float* off[3];
    float* vel[3];
    uint32_t* id;
    float* rho;  // evolved density (continuity model), else null
};

struct FieldsDev {
    float* rho;
    float* p;
    float* s;
    float* inv_rho;
    float* acc[3];
    float* drho;  // optional: drho/dt of the continuity pass
};

// Byte offsets of everything the library keeps in the caller's workspace.
struct Layout {
    size_t err;
    size_t cases;
    size_t items;
    size_t queue;        // item indices in decreasing estimated cost (persistent launches)
    size_t counters;     // one queue counter per neighbour-loop launch of a step
    size_t state[9];     // scratch state for nauticle_step: cell, off[3], vel[3], id, rho
    size_t sort_keys;    // ping-pong keys
    size_t sort_vals;    // ping-pong values
    size_t sort_hist;    // [bins][tiles]
    size_t sort_totals;  // [bins]
    size_t cell_first;   // n_cells_total + 1: first sorted position with key >= c
    size_t pos4;         // float4 per sorted particle: offsets, bits of the cell's x index
    size_t a4;           // float4: offsets, s = p / rho^2
    size_t b4;           // float4: velocity (0 for fixed particles), 1 / rho
    size_t adj4;         // float4: offsets, A_x of the adjoint A = dt (lam_v' + dt lam_x')
    size_t adj2;         // float2: A_y, A_z
    size_t adj4b;        // float4: A, rhobar (after adjoint pass A)
    size_t vr4;          // float4: velocity (0 for fixed), 1 / rho of the step's start (continuity model)
    size_t chmax;        // per-item max |cdot| (Cahn-Hilliard)
    size_t partial;      // per-item FP64 partial sums (2 per item)
    size_t inv_map;      // id -> position map (N u32)
    size_t off0[3];      // offsets at the last build (Verlet steps; N f32 per axis)
    size_t vflag;        // two rebuild words (Verlet steps; one per step parity)
    size_t total;
};

// Packed per-particle arrays in sorted order (workspace).
struct Packed {
    float4* pos4;
    float4* a4;
    float4* b4;
    float4* adj4;
    float4* adj4b;
    uint32_t* cell_first;
    float4* vr4;
    float2* adj2;
};

// Everything derived from a case table.
struct Plan {
    uint64_t fingerprint;
    int32_t n_cases;
    int32_t dim_max;
    uint32_t n_total;
    uint32_t n_cells_total;
    uint32_t n_items;
    uint32_t n_fluid_total;
    int key_bits;
    uint32_t block;          // threads per workgroup = particles per item
    uint32_t persistent;     // neighbour loops as persistent grids
    uint32_t cus;            // compute units of the device (persistent launches)
    uint32_t groups_per_cu;  // persistent groups per compute unit (0: as many as fit)
    uint32_t halo_cap;       // LDS records staged per work item (neighbour loops)
    uint32_t mirror;         // some case has a symmetric axis: the image-aware kernels run
    int32_t model;           // NAUTICLE_MODEL_*, shared by all cases
    Layout L;
    // host copies (for launches that need per-case sizes)
    const CaseDev* host_cases;
};

template <typename T>
inline T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

inline Packed packed(const Plan& P, void* ws)
{
    return Packed{at<float4>(ws, P.L.pos4),  at<float4>(ws, P.L.a4),    at<float4>(ws, P.L.b4),
                  at<float4>(ws, P.L.adj4),  at<float4>(ws, P.L.adj4b), at<uint32_t>(ws, P.L.cell_first),
                  P.L.vr4 ? at<float4>(ws, P.L.vr4) : nullptr, at<float2>(ws, P.L.adj2)};
}

// How a neighbour-loop kernel finds its work items.  A persistent launch
// pulls them from kXcds queues: queue x holds the items an ordinary launch
// gives XCD x (the x-th contiguous slice of the item list, so neighbouring
// tiles share that XCD's L2), in decreasing estimated cost.
struct ItemQueue {
    uint32_t n_items;
    uint32_t persistent;
    const uint32_t* order;  // slice x, position k -> item index, at order[x * ceil(n_items / kXcds) + k]
    uint32_t* counter;      // kXcds counters kCounterStride words apart: the next position in each slice
                            // (zeroed before the launch)
};

constexpr int kMaxBlock = 256;
constexpr int kCounters = 8;  // launches of a sequence with counters of their own
constexpr uint32_t kCounterStride = 32;  // words between two queue counters (one 128-byte line each)

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X, each
// with its own L2.  Tiles are consecutive in space, so giving every XCD one
// contiguous run of tiles keeps neighbouring tiles (which read the same
// neighbour cells) on one L2.  Grid = kXcds * ceil(n_items / kXcds).
constexpr uint32_t kXcds = 8;

inline uint32_t xcd_grid(uint32_t n_items) { return (n_items + kXcds - 1) / kXcds * kXcds; }

__device__ inline uint32_t xcd_item(uint32_t n_items)
{
    const uint32_t per = (n_items + kXcds - 1) / kXcds;
    return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

// Runs body(item) for the items this workgroup owns: its one XCD-mapped
// item (grid launch), or items pulled from the queues (persistent launch):
// first from its own XCD's queue, then, once that is empty, from the
// others' in turn, until all are empty.  Thread 0 claims the next position
// as soon as it has the current item, so the atomic's round trip overlaps
// the item's work; each failed claim moves on to the next queue, so every
// workgroup ends after at most kXcds of them.  Every thread of the block
// must call it; body may contain barriers.
template <typename Body>
__device__ inline void for_each_item(const ItemQueue& Q, uint32_t* s_pos, Body&& body)
{
    const uint32_t per = (Q.n_items + kXcds - 1) / kXcds;
    const uint32_t home = blockIdx.x % kXcds;
    uint32_t tried = 0;  // thread 0: queues found empty
    uint32_t claim = 0;  // thread 0: the claimed position in queue (home + tried) % kXcds
    if (Q.persistent && threadIdx.x == 0) claim = atomicAdd(Q.counter + home * kCounterStride, 1u);
    // one loop for both launch modes, so the body is instantiated once
    for (uint32_t iter = 0;; ++iter) {
        uint32_t ix;
        if (Q.persistent) {
            if (threadIdx.x == 0) {
                uint32_t found = Q.n_items;
                while (tried < kXcds) {
                    const uint32_t x = (home + tried) % kXcds;
                    const uint32_t first = min(x * per, Q.n_items);
                    const uint32_t len = min(per, Q.n_items - first);
                    if (claim < len) {
                        found = Q.order[first + claim];
                        claim = atomicAdd(Q.counter + x * kCounterStride, 1u);  // the next one, ahead
                        break;
                    }
                    if (++tried < kXcds)
                        claim = atomicAdd(Q.counter + ((home + tried) % kXcds) * kCounterStride, 1u);
                }
                *s_pos = found;
            }
            __syncthreads();
            ix = *s_pos;
            __syncthreads();
            if (ix >= Q.n_items) break;
        } else {
            ix = xcd_item(Q.n_items);
            if (iter > 0 || ix >= Q.n_items) break;
        }
        body(ix);
    }
}

// ---- block neighbourhood staging (LDS) ---------------------------------------
// The neighbour loops are bound by the rate at which the vector L1 cache
// serves scattered 16-byte gathers.  A work item's particles are one sorted
// range, in case cells c_lo..c_hi; every neighbour of theirs with cell
// offset (dx, dy, dz) and no periodic fold lies in the cells
// [c_lo - 1, c_hi + 1] shifted by dy rows and dz planes, which is one
// contiguous sorted range per (dy, dz).  Those 3^(dim-1) ranges are copied
// (coalesced) into LDS, and a neighbour j of row r is read from LDS slot
// j + shift[r] when it falls inside the staged range, else from global
// memory (folded neighbours, rows that did not fit).  Which copy is read
// never changes a value.
constexpr uint32_t kHaloRows = 9;
constexpr uint32_t kHaloPad = 16;  // LDS records readable past the staged data

// Records an item may stage for a kernel whose records are na float4s and
// whose LDS budget is `bytes` (the planned need, or what fits).
inline uint32_t halo_records(uint32_t planned, uint32_t na, uint32_t bytes)
{
    const uint32_t fit = bytes / (16u * na) - kHaloPad;
    return planned < fit ? planned : fit;
}
// The search's halo budget: five items of 256 particles per CU.  An item of
// the dense lattice needs ~41 KB for all nine rows; the rows that do not fit
// are read from global memory, which costs less than the occupancy a larger
// halo would take (48 KB: three items per CU, 38 KB: four, 31 KB: five).
constexpr uint32_t kHaloBytes = 31u * 1024u;

struct HaloRows {
    uint32_t lo[kHaloRows];    // staged sorted range [lo, hi) of row r
    uint32_t hi[kHaloRows];    // hi == lo: nothing staged for the row
    int32_t shift[kHaloRows];  // LDS record of sorted index j: j + shift
    uint32_t total;
};

// Row of a (dy, dz) cell offset: r = (dy + 1) + 3 (dz + 1) in 3-D, dy + 1 in 2-D.
template <int DIM>
__device__ inline uint32_t halo_row(int32_t dy, int32_t dz)
{
    return static_cast<uint32_t>(dy + 1) + (DIM == 3 ? 3u * static_cast<uint32_t>(dz + 1) : 0u);
}

// Plans the staged ranges of an item (cap records at most; rows that do not
// fit whole are left to the global path).  Every thread of the block calls it.
template <int DIM>
__device__ inline void halo_plan(const CaseDev& C, const Item& it, const uint32_t* __restrict__ cell,
                                 const uint32_t* __restrict__ cell_first, uint32_t n_total, uint32_t cap,
                                 HaloRows* H)
{
    constexpr uint32_t rows = DIM == 3 ? 9u : 3u;
    if (threadIdx.x < rows) {
        const uint32_t r = threadIdx.x;
        const int64_t dy = static_cast<int64_t>(r % 3u) - 1;
        const int64_t dz = DIM == 3 ? static_cast<int64_t>(r / 3u) - 1 : 0;
        const int64_t S = dy * C.nc[0] + dz * static_cast<int64_t>(C.nc[0]) * C.nc[1];
        const int64_t last = static_cast<int64_t>(C.n_cells) - 1;
        int64_t a = static_cast<int64_t>(min(cell[it.first], C.n_cells - 1)) - 1 + S;
        int64_t b = static_cast<int64_t>(min(cell[it.first + it.count - 1], C.n_cells - 1)) + 1 + S;
        a = a < 0 ? 0 : a;
        b = b > last ? last : b;
        uint32_t lo = 0, hi = 0;
        if (a <= b) {
            lo = min(cell_first[C.cell_base + static_cast<uint32_t>(a)], n_total);
            hi = min(cell_first[C.cell_base + static_cast<uint32_t>(b) + 1u], n_total);
            hi = hi < lo ? lo : hi;
        }
        H->lo[r] = lo;
        H->hi[r] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t used = 0;
        for (uint32_t r = 0; r < rows; ++r) {
            const uint32_t len = H->hi[r] - H->lo[r];
            if (len <= cap - used) {
                H->shift[r] = static_cast<int32_t>(used) - static_cast<int32_t>(H->lo[r]);
                used += len;
            } else {
                H->hi[r] = H->lo[r];
                H->shift[r] = 0;
            }
        }
        H->total = used;
    }
    __syncthreads();
}

// Copies the planned ranges of a per-particle float4 array into `dst`
// (record of sorted index j at dst[j + shift]) and waits for the whole
// block.  Every thread of the block calls it.  Each row is a contiguous run
// in both places, so the copy goes straight from global memory to LDS
// (gfx950 global_load_lds, 16 bytes per lane): the waves share out the
// 64-record pieces of all rows, issue every load before waiting once, and
// the data never passes through registers.
template <int DIM>
__device__ inline void halo_copy(const HaloRows& H, const float4* __restrict__ src, float4* dst)
{
    constexpr uint32_t rows = DIM == 3 ? 9u : 3u;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    uint32_t piece = 0;  // running index over the 64-record pieces of all rows (wave-uniform)
    for (uint32_t r = 0; r < rows; ++r) {
        const uint32_t lo = H.lo[r], len = H.hi[r] - H.lo[r];
        const uint32_t slot = lo + static_cast<uint32_t>(H.shift[r]);  // LDS record of sorted index lo
        for (uint32_t o = 0; o < len; o += 64u, ++piece) {
            if (piece % n_waves != wave) continue;
            if (o + lane < len)
                __builtin_amdgcn_global_load_lds(src + lo + o + lane, (__attribute__((address_space(3))) void*)(dst + slot + o),
                                                 16, 0, 0);
        }
    }
    __syncthreads();  // waits for the loads (vmcnt) before the barrier
}

// Workgroups of a launch of `kernel` (P.block threads, `lds` bytes of
// dynamic LDS): one per item, or for a persistent launch groups_per_cu per
// compute unit, no more than can be resident at once (a group that could
// only start after another had finished would find the queues empty; 0 =
// as many as fit), in whole rounds of kXcds and no more than the items.
uint32_t persistent_groups(const Plan& P, const void* kernel, size_t lds);

inline uint32_t grid_for(const Plan& P, const void* kernel, size_t lds = 0)
{
    return P.persistent ? persistent_groups(P, kernel, lds) : xcd_grid(P.n_items);
}

// Queue for the c-th neighbour-loop launch of a sequence (counter c, reset
// on `s` by this call when the plan is persistent).
hipError_t item_queue(const Plan& P, void* ws, int c, hipStream_t s, ItemQueue* Q);

// ---- launchers (defined in the .hip files) -----------------------------------
// search.hip
hipError_t launch_bin(const Plan& P, void* ws, const float* const pos[3], StateDev st, hipStream_t s);
hipError_t launch_unbin(const Plan& P, void* ws, StateDev st, float* const pos[3], bool by_id, hipStream_t s);
hipError_t launch_gather_id(const Plan& P, void* ws, const uint32_t* id, const float* const g[3],
                            float* const out[3], hipStream_t s);
// mid (optional) is recorded between the sort/reorder and the neighbour lists
hipError_t launch_build_cells(const Plan& P, void* ws, StateDev in, StateDev sorted,
                              const nauticle_cells& cells, hipStream_t s, hipEvent_t mid = nullptr);
hipError_t launch_pack_positions(const Plan& P, void* ws, StateDev sorted, hipStream_t s);
// cell_first (the tiles' particle ranges) from the sorted keys of `cells`
hipError_t launch_cell_first(const Plan& P, void* ws, const nauticle_cells& cells, hipStream_t s);
// sph.hip
hipError_t launch_pack_fields(const Plan& P, void* ws, StateDev sorted, FieldsDev f, hipStream_t s);
// density reads pos4 (written by build_cells or launch_pack_positions) and
// writes the fields plus a4/b4 for the force pass
hipError_t launch_density(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                          FieldsDev f, hipStream_t s);
// continuity reads pos4 and vr4 (launch_pack_continuity) and writes the
// fields plus a4/b4 for the force pass
hipError_t launch_pack_continuity(const Plan& P, void* ws, StateDev sorted, hipStream_t s);
hipError_t launch_continuity(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                             FieldsDev f, hipStream_t s);
// forces read a4/b4 (written by density, continuity or launch_pack_fields);
// the viscous term follows the plan's model
hipError_t launch_forces(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                         FieldsDev f, const StateDev* next, hipStream_t s);
// interact.hip: a pair law (by the plan's model) on the lists of `cells`
struct LawAttrsDev;
hipError_t launch_interact(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                           const LawAttrsDev& attrs, FieldsDev f, const StateDev* next, hipStream_t s);
// ch.hip: n_steps of Example 1b on fixed particles (lists of `cells`)
hipError_t launch_ch_steps(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells, float* c,
                           float* mu, float* cdot, double* clock, int32_t n_steps, hipStream_t s);
// adjoint.hip
hipError_t launch_adjoint(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                          FieldsDev f, const float* const lxn[3], const float* const lvn[3],
                          float* const lx[3], float* const lv[3], double* dnu, double* dc0,
                          hipStream_t s);
// Sets every case's time step from the state's largest fluid speed (CFL),
// writing it into the device case table and advancing the cases' clocks.
hipError_t launch_cfl(const Plan& P, void* ws, StateDev st, double cfl, double* clock, hipStream_t s);
hipError_t launch_position_loss(const Plan& P, void* ws, StateDev a, StateDev b, double* loss,
                                float* const grad[3], hipStream_t s);
// verlet.hip: steps between neighbour builds.  drift completes a step in
// place on the sorted state (velocity, then offset without re-splitting;
// pos4 for the next pair pass; the continuity model's density), records the
// build-time offsets on the first step after a build, and sets rebuild word
// `parity` if some particle has moved beyond its case's lim (clearing the
// other word for the next step).  resplit copies `src` into `dst` with the
// positions re-split into (cell, offset in [0, cs)).
hipError_t launch_verlet_clear(const Plan& P, void* ws, hipStream_t s);
hipError_t launch_verlet_drift(const Plan& P, void* ws, StateDev st, FieldsDev f, bool first, int parity,
                               hipStream_t s);
hipError_t launch_resplit(const Plan& P, void* ws, StateDev src, StateDev dst, hipStream_t s);

// ---- device helpers -----------------------------------------------------------

// Splits an FP32 offset t, measured from the lower face of cell c along one
// axis, into whole cells and a remainder in [0, cs); wraps the cell modulo n
// (periodic shifting on every axis).  Exact same operation order as the
// documented binning rule: k = floor(t * inv_cs); r = fmaf(-k, cs, t); one
// correction of k if r left [0, cs); clamp of a remainder that rounded up to
// cs.  Returns false if |k| would exceed 2^23 (position unrepresentable).
__device__ inline bool split_offset(float t, float cs, float inv_cs, int32_t n, int32_t c,
                                    int32_t* c_out, float* r_out)
{
#pragma clang fp contract(off)
    float q = t * inv_cs;
    float fk = floorf(q);
    bool ok = fabsf(fk) < 8388608.0f;
    if (!ok) fk = 0.0f;
    int32_t k = static_cast<int32_t>(fk);
    float r = __builtin_fmaf(-static_cast<float>(k), cs, t);
    if (r < 0.0f) {
        k -= 1;
        r = __builtin_fmaf(-static_cast<float>(k), cs, t);
    } else if (r >= cs) {
        k += 1;
        r = __builtin_fmaf(-static_cast<float>(k), cs, t);
    }
    if (r < 0.0f) r = 0.0f;
    if (r >= cs) r = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, cs) - 1u);
    int32_t cc = (c + k) % n;
    if (cc < 0) cc += n;
    *c_out = cc;
    *r_out = r;
    return ok;
}

__device__ inline void cell_coords(const CaseDev& C, uint32_t cell, int32_t c[3])
{
    uint32_t nx = static_cast<uint32_t>(C.nc[0]);
    uint32_t ny = static_cast<uint32_t>(C.nc[1]);
    c[0] = static_cast<int32_t>(cell % nx);
    uint32_t r = cell / nx;
    c[1] = static_cast<int32_t>(r % ny);
    c[2] = static_cast<int32_t>(r / ny);
}

__device__ inline void set_error(uint32_t* err, uint32_t bit) { atomicOr(err, bit); }

}  // namespace nau
