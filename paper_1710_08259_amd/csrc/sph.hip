// Interaction sums of the WCSPH step on gfx950: density + Tait equation of
// state, and accelerations with the fused semi-implicit Euler update.
//
// Both passes walk the neighbour lists built by the search (column-major, so
// the 64 lanes of a wave read 64 consecutive words per list row) and gather
// the neighbours' data from sorted SoA arrays, which keeps the gathers
// spatially local (neighbours are within one cell row of each other in
// sorted order) and mostly L2 hits.  Every sum is a gather in a fixed order:
// no atomics, so results are bitwise reproducible.
#include "internal.h"

namespace nau {

struct PairGeom {
    float d[3];  // r_j - r_i (FP32, cell-relative arithmetic)
    float r2;
};

// Decodes a list entry and forms r_j - r_i exactly as the neighbour
// predicate did: d_k = fl32(fl32(off_j,k + delta_k cs_k) - off_i,k).
__device__ inline uint32_t pair_geom(const CaseDev& C, int dim, uint32_t e, uint32_t n_total,
                                     const StateDev& st, const float oi[3], PairGeom* g)
{
#pragma clang fp contract(off)
    uint32_t j = e & kIndexMask;
    if (j >= n_total) j = n_total - 1;  // never for lists built by the search; guards memory
    g->d[2] = 0.0f;
    for (int k = 0; k < 3; ++k) {
        if (k >= dim) break;
        const int32_t dk = static_cast<int32_t>((e >> (NAUTICLE_NBR_INDEX_BITS + 2 * k)) & 3u) - 1;
        const float sh = static_cast<float>(dk) * C.cs[k];
        g->d[k] = (st.off[k][j] + sh) - oi[k];
    }
    float r2 = __builtin_fmaf(g->d[1], g->d[1], g->d[0] * g->d[0]);
    if (dim == 3) r2 = __builtin_fmaf(g->d[2], g->d[2], r2);
    g->r2 = r2;
    return j;
}

// ----------------------------------------------------------------------------
// density + equation of state
// ----------------------------------------------------------------------------
// rho_i = m alpha + sum_j m alpha (1 - q/2)^4 (2q + 1),  q = r_ij / h
// p_i   = B ((rho_i / rho0)^gamma - 1), evaluated as B expm1(gamma log1p(delta))
//         with delta = (rho_i - rho0) / rho0 (no cancellation near rho0)

__global__ void __launch_bounds__(kBlock)
k_density(const CaseDev* __restrict__ cases, const Item* __restrict__ items, StateDev st,
          const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
          uint32_t n_total, FieldsDev f, uint32_t* err)
{
    const Item it = items[blockIdx.x];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const int dim = C.dim;
    float oi[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < dim) oi[k] = st.off[k][i];
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    const float inv_h = C.inv_h;
    float sum = 0.0f;
    for (uint32_t k = 0; k < cnt; ++k) {
        PairGeom g;
        pair_geom(C, dim, nbr[static_cast<size_t>(k) * n_total + i], n_total, st, oi, &g);
        const float q = sqrtf(g.r2) * inv_h;
        const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
        const float t2 = t * t;
        sum = fmaf(t2 * t2, fmaf(2.0f, q, 1.0f), sum);
    }
    const float rho = C.m_alpha * (1.0f + sum);
    const float delta = (rho - C.rho0) * C.inv_rho0;
    const float p = C.B * expm1f(C.gamma * log1pf(delta));
    const float inv_rho = 1.0f / rho;
    f.rho[i] = rho;
    f.p[i] = p;
    f.inv_rho[i] = inv_rho;
    f.s[i] = p * inv_rho * inv_rho;
    if (!isfinite(rho) || !isfinite(p)) set_error(err, kErrNonFinite);
}

hipError_t launch_density(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                          FieldsDev f, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    k_density<<<P.n_items, kBlock, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items), sorted,
                                           cells.nbr, cells.nbr_count, static_cast<uint32_t>(cells.max_nbr),
                                           P.n_total, f, at<uint32_t>(ws, P.L.err));
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// accelerations (+ fused semi-implicit Euler)
// ----------------------------------------------------------------------------
// a_i = -sum_j m (s_i + s_j) F_ij r_ij + sum_j m nu (k_i + k_j) F_ij (v_i - v_j) + g
// with r_ij = -d, F = F_coef (1 - q/2)^3, k = 1/rho.

template <bool kIntegrate>
__global__ void __launch_bounds__(kBlock)
k_forces(const CaseDev* __restrict__ cases, const Item* __restrict__ items, StateDev st,
         const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
         uint32_t n_total, FieldsDev f, StateDev next, uint32_t* err)
{
    const Item it = items[blockIdx.x];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const int dim = C.dim;
    const bool fixed = st.id[i] >= C.n_fluid;
    float oi[3] = {0.0f, 0.0f, 0.0f}, vi[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < dim) {
            oi[k] = st.off[k][i];
            vi[k] = fixed ? 0.0f : st.vel[k][i];
        }
    const float si = f.s[i];
    const float ki = f.inv_rho[i];
    const float inv_h = C.inv_h;
    const float m = C.m;
    const float mnu = C.m * C.nu;
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    float a[3] = {0.0f, 0.0f, 0.0f};
    for (uint32_t k = 0; k < cnt; ++k) {
        PairGeom g;
        const uint32_t j = pair_geom(C, dim, nbr[static_cast<size_t>(k) * n_total + i], n_total, st, oi, &g);
        const float q = sqrtf(g.r2) * inv_h;
        const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
        const float F = C.F_coef * (t * t * t);
        const bool jfixed = st.id[j] >= C.n_fluid;
        // pressure: -m (s_i + s_j) F r_ij = +m (s_i + s_j) F d
        const float cp = m * (si + f.s[j]) * F;
        // viscosity: m nu (k_i + k_j) F (v_i - v_j)
        const float cv = mnu * (ki + f.inv_rho[j]) * F;
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) break;
            const float vj = jfixed ? 0.0f : st.vel[c][j];
            a[c] = fmaf(cp, g.d[c], a[c]);
            a[c] = fmaf(cv, vi[c] - vj, a[c]);
        }
    }
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

hipError_t launch_forces(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                         FieldsDev f, const StateDev* next, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    uint32_t* err = at<uint32_t>(ws, P.L.err);
    const uint32_t mx = static_cast<uint32_t>(cells.max_nbr);
    if (next) {
        k_forces<true><<<P.n_items, kBlock, 0, s>>>(cases, items, sorted, cells.nbr, cells.nbr_count, mx,
                                                    P.n_total, f, *next, err);
    } else {
        StateDev none{};
        k_forces<false><<<P.n_items, kBlock, 0, s>>>(cases, items, sorted, cells.nbr, cells.nbr_count, mx,
                                                     P.n_total, f, none, err);
    }
    return hipGetLastError();
}

}  // namespace nau
