// Reverse mode of one WCSPH step on gfx950 (not in the paper): the
// cotangents of a step's input positions and velocities, and of the
// viscosity nu and sound speed c0, from the cotangents of its outputs.
//
// Two gather passes over the same neighbour lists as the forward step:
//   pass A: sbar, kbar (-> rhobar), viscous part of lam_v, per-particle
//           dnu and dc0 terms;
//   pass B: lam_x (density geometry needs rhobar of the neighbours, so it
//           runs after pass A has finished for every particle).
// Per-case parameter gradients are reduced in FP64 in a fixed order (block
// tree, then items in order), so results are bitwise reproducible.
#include "internal.h"

namespace nau {

namespace {

struct AdjScratch {
    float* A[3];     // dt (lam_v' + dt lam_x'), fluid only
    float* rhobar;
};

__device__ inline void block_reduce2(double a, double b, double* sh_a, double* sh_b, double* out_a,
                                     double* out_b)
{
    sh_a[threadIdx.x] = a;
    sh_b[threadIdx.x] = b;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(s)) {
            sh_a[threadIdx.x] += sh_a[threadIdx.x + s];
            sh_b[threadIdx.x] += sh_b[threadIdx.x + s];
        }
        __syncthreads();
    }
    *out_a = sh_a[0];
    *out_b = sh_b[0];
}

__device__ inline uint32_t adj_pair(const CaseDev& C, int dim, uint32_t e, uint32_t n_total,
                                    const StateDev& st, const float oi[3], float d[3], float* r2)
{
#pragma clang fp contract(off)
    uint32_t j = e & kIndexMask;
    if (j >= n_total) j = n_total - 1;  // never for lists built by the search; guards memory
    d[2] = 0.0f;
    for (int k = 0; k < 3; ++k) {
        if (k >= dim) break;
        const int32_t dk = static_cast<int32_t>((e >> (NAUTICLE_NBR_INDEX_BITS + 2 * k)) & 3u) - 1;
        d[k] = (st.off[k][j] + static_cast<float>(dk) * C.cs[k]) - oi[k];
    }
    float s = __builtin_fmaf(d[1], d[1], d[0] * d[0]);
    if (dim == 3) s = __builtin_fmaf(d[2], d[2], s);
    *r2 = s;
    return j;
}

}  // namespace

// A_i = dt (lam_v'_i + dt lam_x'_i) for fluid particles, 0 for fixed ones.
__global__ void __launch_bounds__(kBlock)
k_adj_prep(const CaseDev* __restrict__ cases, const Item* __restrict__ items, StateDev st,
           const float* __restrict__ lxn0, const float* __restrict__ lxn1, const float* __restrict__ lxn2,
           const float* __restrict__ lvn0, const float* __restrict__ lvn1, const float* __restrict__ lvn2,
           AdjScratch S)
{
    const Item it = items[blockIdx.x];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const bool fixed = st.id[i] >= C.n_fluid;
    const float* lx[3] = {lxn0, lxn1, lxn2};
    const float* lv[3] = {lvn0, lvn1, lvn2};
    for (int k = 0; k < 3; ++k) {
        if (k >= C.dim) break;
        S.A[k][i] = fixed ? 0.0f : C.dt * fmaf(C.dt, lx[k][i], lv[k][i]);
    }
}

// Pass A.
__global__ void __launch_bounds__(kBlock)
k_adj_a(const CaseDev* __restrict__ cases, const Item* __restrict__ items, StateDev st,
        const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
        uint32_t n_total, FieldsDev f, AdjScratch S, const uint32_t* __restrict__ perm,
        const float* __restrict__ lxn0, const float* __restrict__ lxn1, const float* __restrict__ lxn2,
        const float* __restrict__ lvn0, const float* __restrict__ lvn1, const float* __restrict__ lvn2,
        float* lv0, float* lv1, float* lv2, double* __restrict__ partial)
{
    __shared__ double sh_a[kBlock];
    __shared__ double sh_b[kBlock];
    const Item it = items[blockIdx.x];
    const CaseDev& C = cases[it.case_id];
    const bool active = threadIdx.x < it.count;
    double nu_term = 0.0, c0_term = 0.0;
    if (active) {
        const uint32_t i = it.first + threadIdx.x;
        const int dim = C.dim;
        const bool fixed = st.id[i] >= C.n_fluid;
        float oi[3] = {0.0f, 0.0f, 0.0f}, vi[3] = {0.0f, 0.0f, 0.0f}, Ai[3] = {0.0f, 0.0f, 0.0f};
        for (int k = 0; k < 3; ++k)
            if (k < dim) {
                oi[k] = st.off[k][i];
                vi[k] = fixed ? 0.0f : st.vel[k][i];
                Ai[k] = S.A[k][i];
            }
        const float ki = f.inv_rho[i];
        const float m = C.m, mnu = C.m * C.nu;
        uint32_t cnt = nbr_count[i];
        if (cnt > max_nbr) cnt = max_nbr;
        float sbar = 0.0f, kbar = 0.0f, nubar = 0.0f;
        float vv[3] = {0.0f, 0.0f, 0.0f};
        for (uint32_t k = 0; k < cnt; ++k) {
            float d[3], r2;
            const uint32_t j = adj_pair(C, dim, nbr[static_cast<size_t>(k) * n_total + i], n_total, st, oi, d, &r2);
            const float q = sqrtf(r2) * C.inv_h;
            const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
            const float F = C.F_coef * (t * t * t);
            const bool jfixed = st.id[j] >= C.n_fluid;
            float dA[3] = {0.0f, 0.0f, 0.0f}, dv[3] = {0.0f, 0.0f, 0.0f};
            float ddA = 0.0f, dvdA = 0.0f, Aidv = 0.0f;
            for (int c = 0; c < 3; ++c) {
                if (c >= dim) break;
                dA[c] = Ai[c] - S.A[c][j];
                dv[c] = vi[c] - (jfixed ? 0.0f : st.vel[c][j]);
                ddA = fmaf(d[c], dA[c], ddA);
                dvdA = fmaf(dv[c], dA[c], dvdA);
                Aidv = fmaf(Ai[c], dv[c], Aidv);
            }
            // r_ij = -d: sbar_i = -m sum F r_ij.dA = m sum F d.dA
            sbar = fmaf(m * F, ddA, sbar);
            kbar = fmaf(mnu * F, dvdA, kbar);
            const float w = m * (ki + f.inv_rho[j]) * F;
            for (int c = 0; c < 3; ++c)
                if (c < dim) vv[c] = fmaf(C.nu * w, dA[c], vv[c]);
            nubar = fmaf(w, Aidv, nubar);
        }
        const float rho = f.rho[i], p = f.p[i];
        const float inv_rho = ki;
        const float inv_rho2 = inv_rho * inv_rho;
        const float inv_rho3 = inv_rho2 * inv_rho;
        S.rhobar[i] = sbar * (C.gamma * (p + C.B) - 2.0f * p) * inv_rho3 - kbar * inv_rho2;
        (void)rho;
        nu_term = static_cast<double>(nubar);
        c0_term = static_cast<double>(sbar) * (2.0 * static_cast<double>(p) / C.c0) *
                  static_cast<double>(inv_rho2);
        const uint32_t dst = perm[i] < n_total ? perm[i] : i;
        const float* lx[3] = {lxn0, lxn1, lxn2};
        const float* lvn[3] = {lvn0, lvn1, lvn2};
        float* lv[3] = {lv0, lv1, lv2};
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) break;
            const float vh = fmaf(C.dt, lx[c][i], lvn[c][i]);
            lv[c][dst] = fixed ? 0.0f : vh + vv[c];
        }
    }
    double sa, sb;
    block_reduce2(nu_term, c0_term, sh_a, sh_b, &sa, &sb);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa;
        partial[2 * blockIdx.x + 1] = sb;
    }
}

// Pass B.
__global__ void __launch_bounds__(kBlock)
k_adj_b(const CaseDev* __restrict__ cases, const Item* __restrict__ items, StateDev st,
        const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
        uint32_t n_total, FieldsDev f, AdjScratch S, const uint32_t* __restrict__ perm,
        const float* __restrict__ lxn0, const float* __restrict__ lxn1, const float* __restrict__ lxn2,
        float* lx0, float* lx1, float* lx2)
{
    const Item it = items[blockIdx.x];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const int dim = C.dim;
    const bool fixed = st.id[i] >= C.n_fluid;
    const uint32_t dst = perm[i] < n_total ? perm[i] : i;
    float* lx[3] = {lx0, lx1, lx2};
    if (fixed) {
        for (int c = 0; c < 3; ++c)
            if (c < dim) lx[c][dst] = 0.0f;
        return;
    }
    float oi[3] = {0.0f, 0.0f, 0.0f}, vi[3] = {0.0f, 0.0f, 0.0f}, Ai[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < dim) {
            oi[k] = st.off[k][i];
            vi[k] = st.vel[k][i];
            Ai[k] = S.A[k][i];
        }
    const float si = f.s[i], ki = f.inv_rho[i], rbi = S.rhobar[i];
    const float m = C.m, mnu = C.m * C.nu;
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (uint32_t k = 0; k < cnt; ++k) {
        float d[3], r2;
        const uint32_t j = adj_pair(C, dim, nbr[static_cast<size_t>(k) * n_total + i], n_total, st, oi, d, &r2);
        const float r = sqrtf(r2);
        const float q = r * C.inv_h;
        const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
        const float F = C.F_coef * (t * t * t);
        const float Fp_r = r > 0.0f ? C.dF_coef * (t * t) / r : 0.0f;
        const bool jfixed = st.id[j] >= C.n_fluid;
        float dA[3] = {0.0f, 0.0f, 0.0f};
        float ddA = 0.0f, dvdA = 0.0f;
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) break;
            dA[c] = Ai[c] - S.A[c][j];
            const float dv = vi[c] - (jfixed ? 0.0f : st.vel[c][j]);
            ddA = fmaf(d[c], dA[c], ddA);
            dvdA = fmaf(dv, dA[c], dvdA);
        }
        // with r_ij = -d:
        //   density geometry  m F r_ij (rhobar_i + rhobar_j)           = -m F (rb) d
        //   pressure Hessian -m (s_i+s_j) [F dA + (F'/r) r_ij (r_ij.dA)] = -m (s) [F dA + (F'/r) d (d.dA)]
        //   viscous geometry  m nu (k_i+k_j) (F'/r) r_ij (dv.dA)        = -m nu (k) (F'/r) d (dv.dA)
        const float rb = rbi + S.rhobar[j];
        const float cs_ = m * (si + f.s[j]);
        const float ck = mnu * (ki + f.inv_rho[j]);
        const float coef_d = -m * F * rb - cs_ * Fp_r * ddA - ck * Fp_r * dvdA;
        const float coef_a = -cs_ * F;
        for (int c = 0; c < 3; ++c)
            if (c < dim) acc[c] = fmaf(coef_d, d[c], fmaf(coef_a, dA[c], acc[c]));
    }
    const float* lxn[3] = {lxn0, lxn1, lxn2};
    for (int c = 0; c < 3; ++c)
        if (c < dim) lx[c][dst] = lxn[c][i] + acc[c];
}

// Adds each case's sum of item partials (in item order) to out_a / out_b.
__global__ void k_reduce_cases(const CaseDev* __restrict__ cases, int n_cases, const double* __restrict__ partial,
                               double* out_a, double* out_b, int accumulate, double scale_a_by_case)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_cases) return;
    const CaseDev& C = cases[b];
    double sa = 0.0, sb = 0.0;
    for (uint32_t it = C.item_first; it < C.item_first + C.item_count; ++it) {
        sa += partial[2 * it];
        sb += partial[2 * it + 1];
    }
    if (scale_a_by_case != 0.0) {
        const double nf = static_cast<double>(C.n_fluid) * C.dim;
        sa = nf > 0.0 ? sa / nf : 0.0;
    }
    if (out_a) out_a[b] = accumulate ? out_a[b] + sa : sa;
    if (out_b) out_b[b] = accumulate ? out_b[b] + sb : sb;
}

hipError_t launch_adjoint(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                          FieldsDev f, const float* const lxn[3], const float* const lvn[3],
                          float* const lx[3], float* const lv[3], double* dnu, double* dc0,
                          hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    AdjScratch S;
    for (int k = 0; k < 3; ++k) S.A[k] = at<float>(ws, P.L.adj[k]);
    S.rhobar = at<float>(ws, P.L.adj[3]);
    double* partial = at<double>(ws, P.L.partial);
    const uint32_t mx = static_cast<uint32_t>(cells.max_nbr);
    k_adj_prep<<<P.n_items, kBlock, 0, s>>>(cases, items, sorted, lxn[0], lxn[1], lxn[2], lvn[0], lvn[1],
                                            lvn[2], S);
    k_adj_a<<<P.n_items, kBlock, 0, s>>>(cases, items, sorted, cells.nbr, cells.nbr_count, mx, P.n_total, f, S,
                                         cells.perm, lxn[0], lxn[1], lxn[2], lvn[0], lvn[1], lvn[2], lv[0],
                                         lv[1], lv[2], partial);
    k_adj_b<<<P.n_items, kBlock, 0, s>>>(cases, items, sorted, cells.nbr, cells.nbr_count, mx, P.n_total, f, S,
                                         cells.perm, lxn[0], lxn[1], lxn[2], lx[0], lx[1], lx[2]);
    const int nb = (P.n_cases + kBlock - 1) / kBlock;
    k_reduce_cases<<<nb, kBlock, 0, s>>>(cases, P.n_cases, partial, dnu, dc0, 1, 0.0);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// rollout loss between two states matched by id
// ----------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock)
k_inverse_id(const CaseDev* __restrict__ cases, const Item* __restrict__ items, const uint32_t* __restrict__ id,
             uint32_t* __restrict__ inv)
{
    const Item it = items[blockIdx.x];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t p = it.first + threadIdx.x;
    uint32_t k = id[p];
    if (k >= C.n) k = C.n - 1;  // corrupt id: keep the write inside the case
    inv[C.offset + k] = p;
}

__global__ void __launch_bounds__(kBlock)
k_position_loss(const CaseDev* __restrict__ cases, const Item* __restrict__ items, StateDev a, StateDev b,
                const uint32_t* __restrict__ inv_b, float* g0, float* g1, float* g2, double* __restrict__ partial)
{
    __shared__ double sh_a[kBlock];
    __shared__ double sh_b[kBlock];
    const Item it = items[blockIdx.x];
    const CaseDev& C = cases[it.case_id];
    double sq = 0.0;
    if (threadIdx.x < it.count) {
        const uint32_t p = it.first + threadIdx.x;
        const uint32_t ida = a.id[p] < C.n ? a.id[p] : C.n - 1;
        uint32_t q = inv_b[C.offset + ida];
        if (q < C.offset || q >= C.offset + C.n) q = p;  // b is not a permutation of a: guards memory
        const bool fixed = ida >= C.n_fluid;
        int32_t ca[3], cb[3];
        cell_coords(C, a.cell[p], ca);
        cell_coords(C, b.cell[q], cb);
        float* g[3] = {g0, g1, g2};
        const float scale = C.n_fluid > 0 ? 2.0f / (static_cast<float>(C.n_fluid) * C.dim) : 0.0f;
        for (int k = 0; k < 3; ++k) {
            if (k >= C.dim) break;
            int32_t dc = ca[k] - cb[k];
            if (C.periodic[k]) {
                const int32_t n = C.nc[k];
                if (dc > n / 2) dc -= n;
                if (dc < -(n / 2)) dc += n;
            }
            const float delta = static_cast<float>(dc) * C.cs[k] + (a.off[k][p] - b.off[k][q]);
            if (!fixed) sq += static_cast<double>(delta) * delta;
            if (g[k]) g[k][p] = fixed ? 0.0f : scale * delta;
        }
    }
    double sa, sb;
    block_reduce2(sq, 0.0, sh_a, sh_b, &sa, &sb);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa;
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

hipError_t launch_position_loss(const Plan& P, void* ws, StateDev a, StateDev b, double* loss,
                                float* const grad[3], hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    uint32_t* inv = at<uint32_t>(ws, P.L.inv_map);
    double* partial = at<double>(ws, P.L.partial);
    k_inverse_id<<<P.n_items, kBlock, 0, s>>>(cases, items, b.id, inv);
    k_position_loss<<<P.n_items, kBlock, 0, s>>>(cases, items, a, b, inv, grad ? grad[0] : nullptr,
                                                 grad ? grad[1] : nullptr, grad ? grad[2] : nullptr, partial);
    const int nb = (P.n_cases + kBlock - 1) / kBlock;
    k_reduce_cases<<<nb, kBlock, 0, s>>>(cases, P.n_cases, partial, loss, nullptr, 0, 1.0);
    return hipGetLastError();
}

}  // namespace nau
