// Reverse mode of one WCSPH step on gfx950 (not in the paper): the
// cotangents of a step's input positions and velocities, and of the
// viscosity nu and sound speed c0, from the cotangents of its outputs.
//
// Two gather passes over the same neighbour lists as the forward step:
//   pass A: sbar, kbar (-> rhobar), viscous part of lam_v, per-particle
//           dnu and dc0 terms;
//   pass B: lam_x (density geometry needs rhobar of the neighbours, so it
//           runs after pass A has finished for every particle).
// Neighbour data is gathered as float4s in sorted order (offsets + s,
// velocity + 1/rho, A + rhobar).  Per-case parameter gradients are reduced
// in FP64 in a fixed order (block tree, then items in order), so results are
// bitwise reproducible.
#include "internal.h"
#include "pairs.h"

namespace nau {

namespace {

__device__ inline void block_reduce2(double a, double b, double* sh_a, double* sh_b, double* out_a,
                                     double* out_b)
{
    sh_a[threadIdx.x] = a;
    sh_b[threadIdx.x] = b;
    __syncthreads();
    for (int s = static_cast<int>(blockDim.x) / 2; s > 0; s >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(s)) {
            sh_a[threadIdx.x] += sh_a[threadIdx.x + s];
            sh_b[threadIdx.x] += sh_b[threadIdx.x + s];
        }
        __syncthreads();
    }
    *out_a = sh_a[0];
    *out_b = sh_b[0];
}

// r_j - r_i as the neighbour predicate forms it (offsets subtracted first,
// the cell shift added after), from the entry's 6-bit offset code.
__device__ inline float3 adj_d(const CaseDev& C, uint32_t code, const float4& oj, const float4& oi)
{
#pragma clang fp contract(off)
    const float sx = static_cast<float>(static_cast<int32_t>(code & 3u) - 1) * C.cs[0];
    const float sy = static_cast<float>(static_cast<int32_t>((code >> 2) & 3u) - 1) * C.cs[1];
    const float sz = static_cast<float>(static_cast<int32_t>((code >> 4) & 3u) - 1) * C.cs[2];
    return make_float3((oj.x - oi.x) + sx, (oj.y - oi.y) + sy, (oj.z - oi.z) + sz);
}

__device__ inline float adj_r2(const float3& d, int dim)
{
    float r2 = __builtin_fmaf(d.y, d.y, d.x * d.x);
    if (dim == 3) r2 = __builtin_fmaf(d.z, d.z, r2);
    return r2;
}

// Pairs per pipeline stage: three float4 records per neighbour.
constexpr uint32_t kAdjGroup = 4;

}  // namespace

// A_i = dt (lam_v'_i + dt lam_x'_i) for fluid particles, 0 for fixed ones,
// stored with the particle's offsets (from a4) as pass A gathers them: the
// offsets and A_x in one 16-byte record, A_y and A_z in an 8-byte one.  Pass
// A reads neither s_j nor a fourth word of A, so a neighbour takes 10
// registers in its pipeline instead of 12.
__global__ void __launch_bounds__(kMaxBlock)
k_adj_prep(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
           const float* __restrict__ lxn0, const float* __restrict__ lxn1, const float* __restrict__ lxn2,
           const float* __restrict__ lvn0, const float* __restrict__ lvn1, const float* __restrict__ lvn2,
           const float4* __restrict__ a4, float4* __restrict__ adj4, float2* __restrict__ adj2)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const bool fixed = st.id[i] >= C.n_fluid;
    const float* lx[3] = {lxn0, lxn1, lxn2};
    const float* lv[3] = {lvn0, lvn1, lvn2};
    float A[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k) {
        if (k >= C.dim) break;
        A[k] = fixed ? 0.0f : C.dt * fmaf(C.dt, lx[k][i], lv[k][i]);
    }
    const float4 o = a4[i];
    adj4[i] = make_float4(o.x, o.y, o.z, A[0]);
    adj2[i] = make_float2(A[1], A[2]);
}

// Pass A.
__global__ void __launch_bounds__(kMaxBlock)
k_adj_a(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
        const float4* __restrict__ b4, const float4* __restrict__ adj4, const float2* __restrict__ adj2,
        const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
        uint32_t n_total, FieldsDev f, const uint32_t* __restrict__ perm, const float* __restrict__ lxn0,
        const float* __restrict__ lxn1, const float* __restrict__ lxn2, const float* __restrict__ lvn0,
        const float* __restrict__ lvn1, const float* __restrict__ lvn2, float* lv0, float* lv1, float* lv2,
        float4* __restrict__ adj4b, double* __restrict__ partial)
{
    __shared__ double sh_a[kMaxBlock];
    __shared__ double sh_b[kMaxBlock];
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        const bool active = threadIdx.x < it.count;
        double nu_term = 0.0, c0_term = 0.0;
        if (active) {
            const uint32_t i = it.first + threadIdx.x;
            const int dim = C.dim;
            const bool fixed = st.id[i] >= C.n_fluid;
            const float4 oi = adj4[i], bi = b4[i];
            const float2 Ayz = adj2[i];
            const float4 ai = make_float4(oi.x, oi.y, oi.z, 0.0f);
            const float4 Ai = make_float4(oi.w, Ayz.x, Ayz.y, 0.0f);
            const float m = C.m, mnu = C.m * C.nu;
            uint32_t cnt = nbr_count[i];
            if (cnt > max_nbr) cnt = max_nbr;
            float sbar = 0.0f, kbar = 0.0f, nubar = 0.0f;
            float vvx = 0.0f, vvy = 0.0f, vvz = 0.0f;
            const __amdgpu_buffer_rsrc_t ro = float4_rsrc(adj4, n_total), rb = float4_rsrc(b4, n_total);
            const __amdgpu_buffer_rsrc_t r2 = float2_rsrc(adj2, n_total);
            walk_pairs<kAdjGroup, 3>(
                nbr, i, cnt, n_total, dim,
                [&](uint32_t e, float4* v) {
                    v[0] = gather4(ro, e);  // offsets, A_x
                    v[1] = gather4(rb, e);
                    const float2 yz = gather2(r2, e);
                    v[2] = make_float4(yz.x, yz.y, 0.0f, 0.0f);
                },
                [&](uint32_t, const float4* v, uint32_t code) {
                    const float4 aj = make_float4(v[0].x, v[0].y, v[0].z, 0.0f);
                    const float4& bj = v[1];
                    const float4 Aj = make_float4(v[0].w, v[2].x, v[2].y, 0.0f);
                    const float3 d = adj_d(C, code, aj, ai);
                    const float q = pair_sqrt(adj_r2(d, dim)) * C.inv_h;
                    const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
                    const float F = C.F_coef * (t * t * t);  // 0 for padding pairs (t = 0)
                    const float dAx = Ai.x - Aj.x, dAy = Ai.y - Aj.y, dAz = Ai.z - Aj.z;
                    const float dvx = bi.x - bj.x, dvy = bi.y - bj.y, dvz = bi.z - bj.z;
                    const float ddA = fmaf(d.z, dAz, fmaf(d.y, dAy, d.x * dAx));
                    const float dvdA = fmaf(dvz, dAz, fmaf(dvy, dAy, dvx * dAx));
                    const float Aidv = fmaf(Ai.z, dvz, fmaf(Ai.y, dvy, Ai.x * dvx));
                    // r_ij = -d: sbar_i = -m sum F r_ij.dA = m sum F d.dA
                    sbar = fmaf(m * F, ddA, sbar);
                    kbar = fmaf(mnu * F, dvdA, kbar);
                    const float w = m * (bi.w + bj.w) * F;
                    const float wn = C.nu * w;
                    vvx = fmaf(wn, dAx, vvx);
                    vvy = fmaf(wn, dAy, vvy);
                    vvz = fmaf(wn, dAz, vvz);
                    nubar = fmaf(w, Aidv, nubar);
                });
            const float p = f.p[i];
            const float inv_rho2 = bi.w * bi.w;
            const float inv_rho3 = inv_rho2 * bi.w;
            const float rhobar = sbar * (C.gamma * (p + C.B) - 2.0f * p) * inv_rho3 - kbar * inv_rho2;
            adj4b[i] = make_float4(Ai.x, Ai.y, Ai.z, rhobar);
            nu_term = static_cast<double>(nubar);
            c0_term = static_cast<double>(sbar) * (2.0 * static_cast<double>(p) / C.c0) * static_cast<double>(inv_rho2);
            const uint32_t dst = perm[i] < n_total ? perm[i] : i;
            const float* lx[3] = {lxn0, lxn1, lxn2};
            const float* lvn[3] = {lvn0, lvn1, lvn2};
            float* lv[3] = {lv0, lv1, lv2};
            const float vv[3] = {vvx, vvy, vvz};
            for (int c = 0; c < 3; ++c) {
                if (c >= dim) break;
                const float vh = fmaf(C.dt, lx[c][i], lvn[c][i]);
                lv[c][dst] = fixed ? 0.0f : vh + vv[c];
            }
        }
        double sa, sb;
        block_reduce2(nu_term, c0_term, sh_a, sh_b, &sa, &sb);
        if (threadIdx.x == 0) {
            partial[2 * ix] = sa;
            partial[2 * ix + 1] = sb;
        }
    });
}

// Pass B.
__device__ inline void adj_b_particle(const CaseDev& C, uint32_t i, StateDev st, const float4* __restrict__ a4,
                                      const float4* __restrict__ b4, const float4* __restrict__ adj4b,
                                      const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count,
                                      uint32_t max_nbr, uint32_t n_total, const uint32_t* __restrict__ perm,
                                      const float* __restrict__ lxn0, const float* __restrict__ lxn1,
                                      const float* __restrict__ lxn2, float* lx0, float* lx1, float* lx2)
{
    const int dim = C.dim;
    const bool fixed = st.id[i] >= C.n_fluid;
    const uint32_t dst = perm[i] < n_total ? perm[i] : i;
    float* lx[3] = {lx0, lx1, lx2};
    if (fixed) {
        for (int c = 0; c < 3; ++c)
            if (c < dim) lx[c][dst] = 0.0f;
        return;
    }
    const float4 ai = a4[i], bi = b4[i], Ai = adj4b[i];
    const float m = C.m, mnu = C.m * C.nu;
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    float accx = 0.0f, accy = 0.0f, accz = 0.0f;
    const __amdgpu_buffer_rsrc_t ra = float4_rsrc(a4, n_total), rb = float4_rsrc(b4, n_total),
                                 rA = float4_rsrc(adj4b, n_total);
    walk_pairs<kAdjGroup, 3>(
        nbr, i, cnt, n_total, dim,
        [&](uint32_t e, float4* v) {
            v[0] = gather4(ra, e);
            v[1] = gather4(rb, e);
            v[2] = gather4(rA, e);
        },
        [&](uint32_t, const float4* v, uint32_t code) {
            const float4& aj = v[0];
            const float4& bj = v[1];
            const float4& Aj = v[2];
            const float3 d = adj_d(C, code, aj, ai);
            const float r = pair_sqrt(adj_r2(d, dim));
            const float q = r * C.inv_h;
            const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
            // both 0 for padding pairs (t = 0); F'/r with the hardware reciprocal (1 ulp)
            const float F = C.F_coef * (t * t * t);
            const float Fp_r = r > 0.0f ? C.dF_coef * (t * t) * __builtin_amdgcn_rcpf(r) : 0.0f;
            const float dAx = Ai.x - Aj.x, dAy = Ai.y - Aj.y, dAz = Ai.z - Aj.z;
            const float ddA = fmaf(d.z, dAz, fmaf(d.y, dAy, d.x * dAx));
            const float dvdA = fmaf(bi.z - bj.z, dAz, fmaf(bi.y - bj.y, dAy, (bi.x - bj.x) * dAx));
            // with r_ij = -d:
            //   density geometry  m F r_ij (rhobar_i + rhobar_j)             = -m F (rb) d
            //   pressure Hessian -m (s_i+s_j) [F dA + (F'/r) r_ij (r_ij.dA)] = -m (s) [F dA + (F'/r) d (d.dA)]
            //   viscous geometry  m nu (k_i+k_j) (F'/r) r_ij (dv.dA)          = -m nu (k) (F'/r) d (dv.dA)
            const float rb = Ai.w + Aj.w;
            const float cs_ = m * (ai.w + aj.w);
            const float ck = mnu * (bi.w + bj.w);
            const float coef_d = -m * F * rb - cs_ * Fp_r * ddA - ck * Fp_r * dvdA;
            const float coef_a = -cs_ * F;
            accx = fmaf(coef_d, d.x, fmaf(coef_a, dAx, accx));
            accy = fmaf(coef_d, d.y, fmaf(coef_a, dAy, accy));
            accz = fmaf(coef_d, d.z, fmaf(coef_a, dAz, accz));
        });
    const float* lxn[3] = {lxn0, lxn1, lxn2};
    const float acc[3] = {accx, accy, accz};
    for (int c = 0; c < 3; ++c)
        if (c < dim) lx[c][dst] = lxn[c][i] + acc[c];
}

__global__ void __launch_bounds__(kMaxBlock)
k_adj_b(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
        const float4* __restrict__ a4, const float4* __restrict__ b4, const float4* __restrict__ adj4b,
        const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
        uint32_t n_total, const uint32_t* __restrict__ perm, const float* __restrict__ lxn0,
        const float* __restrict__ lxn1, const float* __restrict__ lxn2, float* lx0, float* lx1, float* lx2)
{
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        if (threadIdx.x < it.count)
            adj_b_particle(cases[it.case_id], it.first + threadIdx.x, st, a4, b4, adj4b, nbr, nbr_count, max_nbr,
                           n_total, perm, lxn0, lxn1, lxn2, lx0, lx1, lx2);
    });
}

// Adds each case's sum of its item partials to out_a / out_b: one
// workgroup per case, thread t summing the case's items t, t + blockDim,
// ... in order, then a fixed tree across the threads (the same order on
// every run, and for a case whether it is alone or in a batch).  With
// per_case_mean, out_a gets the sum divided by (n_fluid * dim).
__global__ void __launch_bounds__(kBlock)
k_reduce_cases(const CaseDev* __restrict__ cases, const double* __restrict__ partial, double* out_a, double* out_b,
               int accumulate, int per_case_mean)
{
    __shared__ double sh_a[kBlock];
    __shared__ double sh_b[kBlock];
    const int b = blockIdx.x;
    const CaseDev& C = cases[b];
    double sa = 0.0, sb = 0.0;
    for (uint32_t k = threadIdx.x; k < C.item_count; k += blockDim.x) {
        const uint32_t it = C.item_first + k;
        sa += partial[2 * it];
        sb += partial[2 * it + 1];
    }
    block_reduce2(sa, sb, sh_a, sh_b, &sa, &sb);
    if (threadIdx.x != 0) return;
    if (per_case_mean) {
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
    const Packed pk = packed(P, ws);
    double* partial = at<double>(ws, P.L.partial);
    const uint32_t mx = static_cast<uint32_t>(cells.max_nbr);
    const uint32_t grid = xcd_grid(P.n_items);
    hipError_t e = launch_pack_fields(P, ws, sorted, f, s);
    if (e != hipSuccess) return e;
    k_adj_prep<<<grid, P.block, 0, s>>>(cases, items, P.n_items, sorted, lxn[0], lxn[1], lxn[2], lvn[0], lvn[1],
                                        lvn[2], pk.a4, pk.adj4, pk.adj2);
    ItemQueue Qa, Qb;
    if ((e = item_queue(P, ws, 3, s, &Qa)) != hipSuccess) return e;
    k_adj_a<<<grid_for(P, reinterpret_cast<const void*>(&k_adj_a)), P.block, 0, s>>>(cases, items, Qa, sorted, pk.b4, pk.adj4, pk.adj2, cells.nbr,
                                            cells.nbr_count, mx, P.n_total, f, cells.perm, lxn[0], lxn[1], lxn[2],
                                            lvn[0], lvn[1], lvn[2], lv[0], lv[1], lv[2], pk.adj4b, partial);
    if ((e = item_queue(P, ws, 4, s, &Qb)) != hipSuccess) return e;
    k_adj_b<<<grid_for(P, reinterpret_cast<const void*>(&k_adj_b)), P.block, 0, s>>>(cases, items, Qb, sorted, pk.a4, pk.b4, pk.adj4b, cells.nbr,
                                            cells.nbr_count, mx, P.n_total, cells.perm, lxn[0], lxn[1], lxn[2],
                                            lx[0], lx[1], lx[2]);
    k_reduce_cases<<<P.n_cases, kBlock, 0, s>>>(cases, partial, dnu, dc0, 1, 0);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// rollout loss between two states matched by id
// ----------------------------------------------------------------------------

__global__ void __launch_bounds__(kMaxBlock)
k_inverse_id(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items,
             const uint32_t* __restrict__ id, uint32_t* __restrict__ inv)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t p = it.first + threadIdx.x;
    uint32_t k = id[p];
    if (k >= C.n) k = C.n - 1;  // corrupt id: keep the write inside the case
    inv[C.offset + k] = p;
}

__global__ void __launch_bounds__(kMaxBlock)
k_position_loss(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev a,
                StateDev b, const uint32_t* __restrict__ inv_b, float* g0, float* g1, float* g2,
                double* __restrict__ partial)
{
    __shared__ double sh_a[kMaxBlock];
    __shared__ double sh_b[kMaxBlock];
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;  // uniform over the block
    const Item it = items[ix];
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
        partial[2 * ix] = sa;
        partial[2 * ix + 1] = 0.0;
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
    const uint32_t grid = xcd_grid(P.n_items);
    k_inverse_id<<<grid, P.block, 0, s>>>(cases, items, P.n_items, b.id, inv);
    k_position_loss<<<grid, P.block, 0, s>>>(cases, items, P.n_items, a, b, inv, grad ? grad[0] : nullptr,
                                            grad ? grad[1] : nullptr, grad ? grad[2] : nullptr, partial);
    k_reduce_cases<<<P.n_cases, kBlock, 0, s>>>(cases, partial, loss, nullptr, 0, 1);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// CFL time step
// ----------------------------------------------------------------------------

// partial[2 * item] = the largest speed |v| among the item's fluid particles
// (FP32 |v|, widened; 0 for an item without fluid).
__global__ void __launch_bounds__(kMaxBlock)
k_item_vmax(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
            double* __restrict__ partial)
{
    __shared__ float sh[kMaxBlock];
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;  // uniform over the block
    const Item it = items[ix];
    const CaseDev& C = cases[it.case_id];
    float v = 0.0f;
    if (threadIdx.x < it.count) {
        const uint32_t p = it.first + threadIdx.x;
        if (st.id[p] < C.n_fluid) {
            float s2 = 0.0f;
            for (int k = 0; k < 3; ++k) {
                if (k >= C.dim) break;
                const float vk = st.vel[k][p];
                s2 = fmaf(vk, vk, s2);
            }
            v = __builtin_sqrtf(s2);
        }
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = static_cast<int>(blockDim.x) / 2; s > 0; s >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(s)) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * ix] = static_cast<double>(sh[0]);
        partial[2 * ix + 1] = 0.0;
    }
}

// One workgroup per case: vmax = the largest item maximum (a maximum does
// not depend on the order), dt = cfl h / (c0 + vmax) in FP64, rounded to FP32
// into the device case table (the step's kernels read it there), and the
// case's clock {time, dt} advanced by it.
__global__ void __launch_bounds__(kBlock)
k_cfl_cases(CaseDev* __restrict__ cases, const double* __restrict__ partial, double cfl, double* __restrict__ clock)
{
    __shared__ double sh[kBlock];
    const int b = blockIdx.x;
    CaseDev& C = cases[b];
    double vmax = 0.0;
    for (uint32_t k = threadIdx.x; k < C.item_count; k += blockDim.x) vmax = fmax(vmax, partial[2 * (C.item_first + k)]);
    sh[threadIdx.x] = vmax;
    __syncthreads();
    for (int s = static_cast<int>(blockDim.x) / 2; s > 0; s >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(s)) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const float dt = static_cast<float>(cfl * static_cast<double>(C.h) / (static_cast<double>(C.c0) + sh[0]));
    C.dt = dt;
    clock[2 * b] += static_cast<double>(dt);
    clock[2 * b + 1] = static_cast<double>(dt);
}

hipError_t launch_cfl(const Plan& P, void* ws, StateDev st, double cfl, double* clock, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    double* partial = at<double>(ws, P.L.partial);
    k_item_vmax<<<xcd_grid(P.n_items), P.block, 0, s>>>(cases, at<Item>(ws, P.L.items), P.n_items, st, partial);
    k_cfl_cases<<<P.n_cases, kBlock, 0, s>>>(cases, partial, cfl, clock);
    return hipGetLastError();
}

}  // namespace nau
