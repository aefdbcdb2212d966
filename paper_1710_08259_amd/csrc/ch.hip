// Example 1b on gfx950: the Cahn-Hilliard equation on a fixed particle set
// (a surface in 3-D space) with the SPH Laplacian sph_L0 and the example's
// adaptive time step, every step on the device.
//
// Per step (the example's eq1-eq5 in order):
//   k_ch_mu:    mu_i = c_i^3 - c_i - gamma L(c)_i,
//   k_ch_cdot:  cdot_i = D L(mu)_i,  c_i += dt cdot_i,  max |cdot| per item,
//   k_ch_clock: max over the case's items; time += dt;
//               dt = fac min(1 / max|cdot|, gamma / (2h)^2),
// with L(A)_i = 2 V sum_j (A_i - A_j) F_ij (eq. diffop3 as the example
// discretises it; V = m / rho0; F with the kernel normalised in 2-D).  The
// particles never move, so the neighbour lists are built once by the caller
// (the paper runs the search only when the layout changes).  Both passes
// gather one float4 per pair, (offsets, field), with the pipelined walk of
// pairs.h.
#include "internal.h"
#include "pairs.h"

namespace nau {

// ~12 neighbours per particle on the surface: groups of 4 pairs per stage
constexpr uint32_t kChGroup = 4;

// (offsets, c) of every sorted particle.
__global__ void __launch_bounds__(kMaxBlock)
k_ch_pack(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
          const float* __restrict__ c, float4* __restrict__ rc)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    float o[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < C.dim) o[k] = st.off[k][i];
    rc[i] = make_float4(o[0], o[1], o[2], c[i]);
}

// 2 V sum_j (A_i - A_j) F_ij over i's list, (offsets, A) records in `rec`.
template <bool kMirror, uint32_t G>
__device__ inline float ch_laplacian(const CaseDev& C, const ShiftTable& tab, uint32_t i, const float4& me,
                                     StateDev st, const float4* __restrict__ rec, const uint32_t* __restrict__ nbr,
                                     uint32_t cnt, uint32_t n_total)
{
    ImageFrame M{};
    if constexpr (kMirror) M = image_frame(C, min(st.cell[i], C.n_cells - 1));
    const __amdgpu_buffer_rsrc_t q = float4_rsrc(rec, n_total);
    const float inv_h = C.inv_h;
    float sum = 0.0f;
    walk_pairs<G, 1>(
        nbr, i, cnt, n_total, C.dim, [&](uint32_t e, float4* v) { v[0] = gather4(q, e); },
        [&](uint32_t, const float4* v, uint32_t code) {
            float3 d, sg;
            if constexpr (kMirror) d = pair_d_img(tab.v[code], code, M, v[0].x, v[0].y, v[0].z, me.x, me.y, me.z, &sg);
            else d = pair_d(tab.v[code], v[0].x, v[0].y, v[0].z, me.x, me.y, me.z);
            const float qq = pair_sqrt(pair_r2(d, C.dim)) * inv_h;
            const float t = fmaxf(1.0f - 0.5f * qq, 0.0f);
            sum = fmaf(me.w - v[0].w, t * t * t, sum);  // F / F_coef; 0 for padding pairs
        });
    return 2.0f * C.m * C.inv_rho0 * C.F_coef * sum;
}

template <bool kMirror, uint32_t G>
__global__ void __launch_bounds__(kMaxBlock)
k_ch_mu(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
        const float4* __restrict__ rc, float4* __restrict__ rm, const uint32_t* __restrict__ nbr,
        const uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total, float* __restrict__ mu,
        uint32_t* err)
{
    __shared__ ShiftTable tab;
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        fill_shift_table(C, &tab);
        if (threadIdx.x < it.count) {
            const uint32_t i = it.first + threadIdx.x;
            const float4 me = rc[i];
            uint32_t cnt = nbr_count[i];
            if (cnt > max_nbr) cnt = max_nbr;
            const float L = ch_laplacian<kMirror, G>(C, tab, i, me, st, rc, nbr, cnt, n_total);
            const float c = me.w;
            const float m = fmaf(c * c, c, -c) - C.law[1] * L;
            rm[i] = make_float4(me.x, me.y, me.z, m);
            if (mu) mu[i] = m;
            if (!isfinite(m)) set_error(err, kErrNonFinite);
        }
    });
}

template <bool kMirror, uint32_t G>
__global__ void __launch_bounds__(kMaxBlock)
k_ch_cdot(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
          float4* __restrict__ rc, const float4* __restrict__ rm, const uint32_t* __restrict__ nbr,
          const uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total, float* __restrict__ c_out,
          float* __restrict__ cdot_out, const double* __restrict__ clock, float* __restrict__ item_max,
          uint32_t* err)
{
    __shared__ ShiftTable tab;
    __shared__ uint32_t s_pos;
    __shared__ float s_max[kMaxBlock / 64];
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        fill_shift_table(C, &tab);
        float a = 0.0f;  // |cdot| of this lane (0 for idle lanes)
        if (threadIdx.x < it.count) {
            const uint32_t i = it.first + threadIdx.x;
            const float4 me = rm[i];
            uint32_t cnt = nbr_count[i];
            if (cnt > max_nbr) cnt = max_nbr;
            const float cd = C.law[0] * ch_laplacian<kMirror, G>(C, tab, i, me, st, rm, nbr, cnt, n_total);
            const float dt = static_cast<float>(clock[2 * it.case_id + 1]);
            const float4 own = rc[i];  // only particle i's own record: no other lane reads it here
            const float cn = fmaf(dt, cd, own.w);
            rc[i] = make_float4(own.x, own.y, own.z, cn);
            c_out[i] = cn;
            if (cdot_out) cdot_out[i] = cd;
            a = fabsf(cd);
            if (!isfinite(cn)) set_error(err, kErrNonFinite);
        }
        // the item's maximum: within each wave, then across the waves in
        // LDS; one plain store per item (no atomics on a shared address)
        for (int off = 32; off > 0; off >>= 1) a = fmaxf(a, __shfl_xor(a, off));
        if ((threadIdx.x & 63u) == 0u) s_max[threadIdx.x >> 6] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = 0.0f;
            for (uint32_t w = 0; w < blockDim.x / 64; ++w) m = fmaxf(m, s_max[w]);
            item_max[ix] = m;
        }
        __syncthreads();  // s_max is reused by the next item
    });
}

// eq1 and eq5, one workgroup per case: the maximum of |cdot| over the
// case's items, then time += dt; dt = fac min(1 / max|cdot|, dt_g).
__global__ void __launch_bounds__(kBlock)
k_ch_clock(const CaseDev* __restrict__ cases, double* __restrict__ clock, const float* __restrict__ item_max)
{
    __shared__ float s_max[kBlock / 64];
    const uint32_t b = blockIdx.x;
    const CaseDev& C = cases[b];
    float m = 0.0f;
    for (uint32_t k = threadIdx.x; k < C.item_count; k += blockDim.x) m = fmaxf(m, item_max[C.item_first + k]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63u) == 0u) s_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mx = 0.0f;
        for (uint32_t w = 0; w < blockDim.x / 64; ++w) mx = fmaxf(mx, s_max[w]);
        const double dt_g = static_cast<double>(C.law[3]);
        const double lim = mx > 0.0f ? 1.0 / static_cast<double>(mx) : dt_g;
        clock[2 * b] += clock[2 * b + 1];
        clock[2 * b + 1] = static_cast<double>(C.law[2]) * (lim < dt_g ? lim : dt_g);
    }
}

hipError_t launch_ch_steps(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells, float* c,
                           float* mu, float* cdot, double* clock, int32_t n_steps, hipStream_t s)
{
    if (P.n_items == 0 || n_steps <= 0) return hipSuccess;
    const Packed pk = packed(P, ws);
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    uint32_t* err = at<uint32_t>(ws, P.L.err);
    float* item_max = at<float>(ws, P.L.chmax);
    const uint32_t mx = static_cast<uint32_t>(cells.max_nbr);
    k_ch_pack<<<xcd_grid(P.n_items), P.block, 0, s>>>(cases, items, P.n_items, sorted, c, pk.a4);
    hipError_t e = hipGetLastError();
    auto kmu = P.mirror ? k_ch_mu<true, kChGroup> : k_ch_mu<false, kChGroup>;
    auto kcd = P.mirror ? k_ch_cdot<true, kChGroup> : k_ch_cdot<false, kChGroup>;
    for (int32_t step = 0; step < n_steps && e == hipSuccess; ++step) {
        ItemQueue Q;
        if ((e = item_queue(P, ws, 6, s, &Q)) != hipSuccess) break;
        kmu<<<grid_for(P, reinterpret_cast<const void*>(kmu)), P.block, 0, s>>>(cases, items, Q, sorted, pk.a4, pk.b4, cells.nbr, cells.nbr_count, mx,
                                            P.n_total, mu, err);
        if ((e = item_queue(P, ws, 7, s, &Q)) != hipSuccess) break;
        kcd<<<grid_for(P, reinterpret_cast<const void*>(kcd)), P.block, 0, s>>>(cases, items, Q, sorted, pk.a4, pk.b4, cells.nbr, cells.nbr_count, mx,
                                            P.n_total, c, cdot, clock, item_max, err);
        k_ch_clock<<<P.n_cases, kBlock, 0, s>>>(cases, clock, item_max);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace nau
