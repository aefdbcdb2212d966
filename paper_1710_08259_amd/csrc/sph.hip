// Interaction sums of the WCSPH step on gfx950: density + Tait equation of
// state, and accelerations with the fused semi-implicit Euler update.
//
// Both passes walk the neighbour lists built by the search (16-byte chunks of
// four entries, so the 64 lanes of a wave read 1 KB contiguous per chunk
// row) with the pipelined walk of pairs.h.  Each neighbour costs one float4
// gather in the density pass (offsets) and two in the force pass (offsets +
// s, velocity + 1/rho), from arrays in sorted order, so the gathers of a wave
// stay within a few cells.  Every sum is taken in list order: no atomics, so
// results are bitwise reproducible.
#include "internal.h"
#include "pairs.h"

namespace nau {

constexpr uint32_t kForceGroup = 8;

// ----------------------------------------------------------------------------
// density + equation of state (arithmetic in pairs.h)
// ----------------------------------------------------------------------------
// rho_i = m alpha + sum_j m alpha (1 - q/2)^4 (2q + 1),  q = r_ij / h
// p_i   = B ((rho_i / rho0)^gamma - 1), evaluated as B expm1(gamma log1p(delta))
//         with delta = (rho_i - rho0) / rho0 (no cancellation near rho0)
// Also packs (offsets, s) and (velocity, 1/rho) for the force pass; fixed
// particles get velocity 0 there.

__device__ inline void density_particle(const CaseDev& C, const ShiftTable& tab, uint32_t i, StateDev st,
                                        const float4* __restrict__ pos4, const uint32_t* __restrict__ nbr,
                                        const uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total,
                                        FieldsDev f, float4* __restrict__ a4, float4* __restrict__ b4, uint32_t* err)
{
    const float4 me = pos4[i];
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    const __amdgpu_buffer_rsrc_t rpos = float4_rsrc(pos4, n_total);
    auto gather = [&](uint32_t e, float4* v) { v[0] = gather4(rpos, e); };
    const float sum = C.dim == 3 ? density_sum<3>(C, tab, i, me, nbr, cnt, n_total, gather)
                                 : density_sum<2>(C, tab, i, me, nbr, cnt, n_total, gather);
    density_finish(C, i, sum, me, st, f, a4, b4, err);
}

__global__ void __launch_bounds__(kMaxBlock)
k_density(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
          const float4* __restrict__ pos4, const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count,
          uint32_t max_nbr, uint32_t n_total, FieldsDev f, float4* __restrict__ a4, float4* __restrict__ b4,
          uint32_t* err)
{
    __shared__ ShiftTable tab;
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        fill_shift_table(C, &tab);
        if (threadIdx.x < it.count)
            density_particle(C, tab, it.first + threadIdx.x, st, pos4, nbr, nbr_count, max_nbr, n_total, f, a4, b4,
                             err);
    });
}

hipError_t launch_density(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                          FieldsDev f, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const Packed pk = packed(P, ws);
    ItemQueue Q;
    hipError_t e = item_queue(P, ws, 1, s, &Q);
    if (e != hipSuccess) return e;
    k_density<<<grid_for(P), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items), Q, sorted,
                                              pk.pos4, cells.nbr, cells.nbr_count,
                                              static_cast<uint32_t>(cells.max_nbr), P.n_total, f, pk.a4, pk.b4,
                                              at<uint32_t>(ws, P.L.err));
    return hipGetLastError();
}

// Packs (offsets, s) and (velocity, 1/rho) from caller-provided fields, for
// a force pass that does not follow a density pass on this workspace.
__global__ void __launch_bounds__(kMaxBlock)
k_pack_fields(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
              FieldsDev f, float4* __restrict__ a4, float4* __restrict__ b4)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const bool fixed = st.id[i] >= C.n_fluid;
    float o[3] = {0.0f, 0.0f, 0.0f}, v[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < C.dim) {
            o[k] = st.off[k][i];
            v[k] = fixed ? 0.0f : st.vel[k][i];
        }
    a4[i] = make_float4(o[0], o[1], o[2], f.s[i]);
    b4[i] = make_float4(v[0], v[1], v[2], f.inv_rho[i]);
}

hipError_t launch_pack_fields(const Plan& P, void* ws, StateDev sorted, FieldsDev f, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const Packed pk = packed(P, ws);
    k_pack_fields<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                         P.n_items, sorted, f, pk.a4, pk.b4);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// accelerations (+ fused semi-implicit Euler)
// ----------------------------------------------------------------------------
// a_i = -sum_j m (s_i + s_j) F_ij r_ij + sum_j m nu (k_i + k_j) F_ij (v_i - v_j) + g
// with r_ij = -d, F = F_coef (1 - q/2)^3, k = 1/rho.

template <bool kIntegrate>
__device__ inline void forces_particle(const CaseDev& C, const ShiftTable& tab, uint32_t i, StateDev st,
                                       const float4* __restrict__ a4, const float4* __restrict__ b4,
                                       const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count,
                                       uint32_t max_nbr, uint32_t n_total, FieldsDev f, StateDev next, uint32_t* err)
{
    const int dim = C.dim;
    const float4 ai4 = a4[i];
    const float4 bi4 = b4[i];
    const float inv_h = C.inv_h;
    const float m = C.m;
    const float mnu = C.m * C.nu;
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    const __amdgpu_buffer_rsrc_t ra = float4_rsrc(a4, n_total), rb = float4_rsrc(b4, n_total);
    walk_pairs<kForceGroup, 2>(
        nbr, i, cnt, n_total, dim,
        [&](uint32_t e, float4* v) {
            v[0] = gather4(ra, e);
            v[1] = gather4(rb, e);
        },
        [&](uint32_t, const float4* v, uint32_t code) {
            const float4& aj = v[0];
            const float4& bj = v[1];
            const float3 d = pair_d(tab.v[code], aj.x, aj.y, aj.z, ai4.x, ai4.y, ai4.z);
            const float q = pair_sqrt(pair_r2(d, dim)) * inv_h;
            const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
            const float F = C.F_coef * (t * t * t);  // 0 for padding pairs (t = 0)
            // pressure: -m (s_i + s_j) F r_ij = +m (s_i + s_j) F d
            const float cp = m * (ai4.w + aj.w) * F;
            // viscosity: m nu (k_i + k_j) F (v_i - v_j)
            const float cv = mnu * (bi4.w + bj.w) * F;
            ax = fmaf(cp, d.x, fmaf(cv, bi4.x - bj.x, ax));
            ay = fmaf(cp, d.y, fmaf(cv, bi4.y - bj.y, ay));
            az = fmaf(cp, d.z, fmaf(cv, bi4.z - bj.z, az));
        });
    const bool fixed = st.id[i] >= C.n_fluid;
    float a[3] = {ax, ay, az};
    const float vi[3] = {bi4.x, bi4.y, bi4.z};
    const float oi[3] = {ai4.x, ai4.y, ai4.z};
    bool finite = true;
    for (int c = 0; c < 3; ++c) {
        if (c >= dim) break;
        a[c] = fixed ? 0.0f : a[c] + C.g[c];
        f.acc[c][i] = a[c];
        finite &= isfinite(a[c]);
    }
    if (!finite) set_error(err, kErrNonFinite);
    if constexpr (kIntegrate) {
        // v' = v + dt a; offset t = off + dt v' re-split into (cell, offset)
        int32_t cc[3] = {0, 0, 0};
        cell_coords(C, st.cell[i], cc);
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) break;
            float vn = fixed ? 0.0f : fmaf(C.dt, a[c], vi[c]);
            float on = oi[c];
            int32_t cn = cc[c];
            if (!fixed) {
                const float tpos = fmaf(C.dt, vn, oi[c]);
                ok &= split_offset(tpos, C.cs[c], C.inv_cs[c], C.nc[c], cc[c], &cn, &on);
            }
            next.vel[c][i] = vn;
            next.off[c][i] = on;
            cc[c] = cn;
        }
        if (!ok) set_error(err, kErrOutOfDomain);
        next.cell[i] = static_cast<uint32_t>(cc[0]) +
                       static_cast<uint32_t>(C.nc[0]) *
                           (static_cast<uint32_t>(cc[1]) + static_cast<uint32_t>(C.nc[1]) * static_cast<uint32_t>(cc[2]));
        next.id[i] = st.id[i];
    }
}

template <bool kIntegrate>
__global__ void __launch_bounds__(kMaxBlock)
k_forces(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
         const float4* __restrict__ a4, const float4* __restrict__ b4, const uint32_t* __restrict__ nbr,
         const uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total, FieldsDev f, StateDev next,
         uint32_t* err)
{
    __shared__ ShiftTable tab;
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        fill_shift_table(C, &tab);
        if (threadIdx.x < it.count)
            forces_particle<kIntegrate>(C, tab, it.first + threadIdx.x, st, a4, b4, nbr, nbr_count, max_nbr, n_total,
                                        f, next, err);
    });
}

hipError_t launch_forces(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                         FieldsDev f, const StateDev* next, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    uint32_t* err = at<uint32_t>(ws, P.L.err);
    const Packed pk = packed(P, ws);
    const uint32_t mx = static_cast<uint32_t>(cells.max_nbr);
    ItemQueue Q;
    hipError_t e = item_queue(P, ws, 2, s, &Q);
    if (e != hipSuccess) return e;
    if (next) {
        k_forces<true><<<grid_for(P), P.block, 0, s>>>(cases, items, Q, sorted, pk.a4, pk.b4, cells.nbr,
                                                       cells.nbr_count, mx, P.n_total, f, *next, err);
    } else {
        StateDev none{};
        k_forces<false><<<grid_for(P), P.block, 0, s>>>(cases, items, Q, sorted, pk.a4, pk.b4, cells.nbr,
                                                        cells.nbr_count, mx, P.n_total, f, none, err);
    }
    return hipGetLastError();
}

}  // namespace nau
