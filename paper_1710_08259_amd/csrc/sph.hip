// Interaction sums of the WCSPH step on gfx950: density + Tait equation of
// state (or, in Example 1a's model, the continuity equation + the linear
// equation of state), and accelerations with the fused semi-implicit Euler
// update.
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

// Pairs per pipeline stage of the pair passes: 8 in 3-D (~57 neighbours per
// particle); 4 in 2-D, where lists are short (~12-25 entries) and the
// smaller stages leave registers for more resident waves to hide the
// walk's latency.  The 3-D density sum, one record per neighbour, takes 12
// where lists are long (three waves per SIMD with 24 gathers in flight each
// beat four with 16); where they are short, padding to whole stages of 12
// costs more than that gains.  The order of every sum does not depend on it.
constexpr uint32_t kGroup3 = 8;
constexpr uint32_t kGroup2 = 4;
constexpr uint32_t kDensityGroup3Long = 12;
constexpr double kLongList = 48.0;  // expected neighbours per particle

// Expected neighbours per particle at a case's mean number density: the
// particles per cell times the ball of radius 2h over the cell (3-D).
inline double expected_neighbours_3d(const CaseDev& C)
{
    const double r = std::sqrt(static_cast<double>(C.R2));
    const double cell = static_cast<double>(C.cs[0]) * C.cs[1] * C.cs[2];
    return static_cast<double>(C.n) / C.n_cells * (4.0 / 3.0 * M_PI * r * r * r) / cell;
}

// ----------------------------------------------------------------------------
// density + equation of state (arithmetic in pairs.h)
// ----------------------------------------------------------------------------
// rho_i = m alpha + sum_j m alpha (1 - q/2)^4 (2q + 1),  q = r_ij / h
// p_i   = B ((rho_i / rho0)^gamma - 1), evaluated as B expm1(gamma log1p(delta))
//         with delta = (rho_i - rho0) / rho0 (no cancellation near rho0)
// Also packs (offsets, s) and (velocity, 1/rho) for the force pass; fixed
// particles get velocity 0 there.

template <bool kMirror, uint32_t G>
__device__ inline void density_particle(const CaseDev& C, const ShiftTable& tab, uint32_t i, StateDev st,
                                        const float4* __restrict__ pos4, const uint32_t* __restrict__ nbr,
                                        const uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total,
                                        FieldsDev f, float4* __restrict__ a4, float4* __restrict__ b4, uint32_t* err)
{
    const float4 me = pos4[i];
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    ImageFrame M{};
    if constexpr (kMirror) M = image_frame(C, min(st.cell[i], C.n_cells - 1));
    const __amdgpu_buffer_rsrc_t rpos = float4_rsrc(pos4, n_total);
    auto gather = [&](uint32_t e, float4* v) { v[0] = gather4(rpos, e); };
    const float sum = C.dim == 3 ? density_sum<3, kMirror, G>(C, tab, M, i, me, nbr, cnt, n_total, gather)
                                 : density_sum<2, kMirror, G>(C, tab, M, i, me, nbr, cnt, n_total, gather);
    density_finish(C, i, sum, me, st, f, a4, b4, err);
}

template <bool kMirror, uint32_t G>
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
            density_particle<kMirror, G>(C, tab, it.first + threadIdx.x, st, pos4, nbr, nbr_count, max_nbr, n_total,
                                         f, a4, b4, err);
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
    bool long_lists = false;
    for (int b = 0; b < P.n_cases && P.dim_max == 3; ++b)
        long_lists |= expected_neighbours_3d(P.host_cases[b]) >= kLongList;
    auto k3 = long_lists ? (P.mirror ? k_density<true, kDensityGroup3Long> : k_density<false, kDensityGroup3Long>)
                         : (P.mirror ? k_density<true, kGroup3> : k_density<false, kGroup3>);
    auto kern = P.dim_max == 3 ? k3
                               : (P.mirror ? k_density<true, kGroup2> : k_density<false, kGroup2>);
    kern<<<grid_for(P, reinterpret_cast<const void*>(kern)), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items), Q, sorted, pk.pos4,
                                         cells.nbr, cells.nbr_count, static_cast<uint32_t>(cells.max_nbr), P.n_total,
                                         f, pk.a4, pk.b4, at<uint32_t>(ws, P.L.err));
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// continuity + linear equation of state (Example 1a's model)
// ----------------------------------------------------------------------------
// drho_i/dt = -rho_i sum_j (v_j - v_i) . grad_i W_ij m / rho_j
//           = m rho_i sum_j F_ij ((v_j - v_i) . d) / rho_j      (grad_i W = -F d)
// then rho_i' = rho_i + dt drho_i, p_i = c^2 (rho_i' - rho0), s = p/rho'^2,
// 1/rho'; packs (offsets, s) and (velocity, 1/rho') for the force pass.
// Every neighbour value read is from the step's start (vr4), so the sum
// for all particles is finished before any density changes.

// (velocity, 0 for fixed particles; 1/rho) of the sorted state, gathered by
// the continuity pass.
__global__ void __launch_bounds__(kMaxBlock)
k_pack_continuity(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
                  float4* __restrict__ vr4)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const bool fixed = st.id[i] >= C.n_fluid;
    float v[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < C.dim && !fixed) v[k] = st.vel[k][i];
    vr4[i] = make_float4(v[0], v[1], v[2], 1.0f / st.rho[i]);
}

hipError_t launch_pack_continuity(const Plan& P, void* ws, StateDev sorted, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const Packed pk = packed(P, ws);
    k_pack_continuity<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                             P.n_items, sorted, pk.vr4);
    return hipGetLastError();
}

template <bool kMirror, uint32_t G>
__device__ inline void continuity_particle(const CaseDev& C, const ShiftTable& tab, uint32_t i, StateDev st,
                                           const float4* __restrict__ pos4, const float4* __restrict__ vr4,
                                           const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count,
                                           uint32_t max_nbr, uint32_t n_total, FieldsDev f, float4* __restrict__ a4,
                                           float4* __restrict__ b4, uint32_t* err)
{
    const int dim = C.dim;
    const float4 me = pos4[i];
    const float4 vi = vr4[i];
    const float inv_h = C.inv_h;
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    ImageFrame M{};
    if constexpr (kMirror) M = image_frame(C, min(st.cell[i], C.n_cells - 1));
    float sum = 0.0f;
    const __amdgpu_buffer_rsrc_t rp = float4_rsrc(pos4, n_total), rv = float4_rsrc(vr4, n_total);
    walk_pairs<G, 2>(
        nbr, i, cnt, n_total, dim,
        [&](uint32_t e, float4* v) {
            v[0] = gather4(rp, e);
            v[1] = gather4(rv, e);
        },
        [&](uint32_t, const float4* v, uint32_t code) {
            const float4& oj = v[0];
            const float4& vj = v[1];
            float3 d, sg = make_float3(1.0f, 1.0f, 1.0f);
            if constexpr (kMirror) d = pair_d_img(tab.v[code], code, M, oj.x, oj.y, oj.z, me.x, me.y, me.z, &sg);
            else d = pair_d(tab.v[code], oj.x, oj.y, oj.z, me.x, me.y, me.z);
            const float q = pair_sqrt(pair_r2(d, dim)) * inv_h;
            const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
            const float F = t * t * t;  // times F_coef after the sum; 0 for padding pairs
            // (v_j - v_i) . d with the image's velocity
            const float dvd = fmaf(fmaf(sg.z, vj.z, -vi.z), d.z,
                                   fmaf(fmaf(sg.y, vj.y, -vi.y), d.y, fmaf(sg.x, vj.x, -vi.x) * d.x));
            sum = fmaf(F * dvd, vj.w, sum);
        });
    const float rho = st.rho[i];
    const float drho = C.m * C.F_coef * rho * sum;
    const float rn = fmaf(C.dt, drho, rho);
    const float p = C.c2 * (rn - C.rho0);
    const float inv_rho = 1.0f / rn;
    const float s = p * inv_rho * inv_rho;
    f.rho[i] = rn;
    f.p[i] = p;
    f.s[i] = s;
    f.inv_rho[i] = inv_rho;
    if (f.drho) f.drho[i] = drho;
    a4[i] = make_float4(me.x, me.y, me.z, s);
    b4[i] = make_float4(vi.x, vi.y, vi.z, inv_rho);
    if (!isfinite(rn) || !isfinite(drho)) set_error(err, kErrNonFinite);
}

template <bool kMirror, uint32_t G>
__global__ void __launch_bounds__(kMaxBlock)
k_continuity(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st,
             const float4* __restrict__ pos4, const float4* __restrict__ vr4, const uint32_t* __restrict__ nbr,
             const uint32_t* __restrict__ nbr_count, uint32_t max_nbr, uint32_t n_total, FieldsDev f,
             float4* __restrict__ a4, float4* __restrict__ b4, uint32_t* err)
{
    __shared__ ShiftTable tab;
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        fill_shift_table(C, &tab);
        if (threadIdx.x < it.count)
            continuity_particle<kMirror, G>(C, tab, it.first + threadIdx.x, st, pos4, vr4, nbr, nbr_count, max_nbr,
                                         n_total, f, a4, b4, err);
    });
}

hipError_t launch_continuity(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells, FieldsDev f,
                             hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    const Packed pk = packed(P, ws);
    ItemQueue Q;
    hipError_t e = item_queue(P, ws, 1, s, &Q);
    if (e != hipSuccess) return e;
    auto kern = P.dim_max == 3 ? (P.mirror ? k_continuity<true, kGroup3> : k_continuity<false, kGroup3>)
                               : (P.mirror ? k_continuity<true, kGroup2> : k_continuity<false, kGroup2>);
    kern<<<grid_for(P, reinterpret_cast<const void*>(kern)), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items), Q, sorted, pk.pos4,
                                         pk.vr4, cells.nbr, cells.nbr_count, static_cast<uint32_t>(cells.max_nbr),
                                         P.n_total, f, pk.a4, pk.b4, at<uint32_t>(ws, P.L.err));
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
// a_i = -sum_j m (s_i + s_j) F_ij r_ij + viscous term + g, with r_ij = -d,
// F = F_coef (1 - q/2)^3, k = 1/rho; the viscous term of
//   the summation model (Morris): sum_j m nu (k_i + k_j) F_ij (v_i - v_j);
//   Example 1a's model (artificial viscosity, eq. SPH_fluid_momentum):
//     -sum_j Pi_ij m F_ij r_ij,  Pi_ij = -alpha c h w / (rho_i r^2) if
//     w = (v_i - v_j) . r_ij < 0, else 0 (rho_i, as printed).  A coincident
//     pair has w = 0: no term (the select never multiplies 0 by 1/0).
// For an image neighbour (kMirror) v_j is the reflected velocity.

template <bool kIntegrate, int kModel, bool kMirror, uint32_t G>
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
    const float cav = C.av_coef * bi4.w;  // alpha c h m / rho_i
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    ImageFrame M{};
    if constexpr (kMirror) M = image_frame(C, min(st.cell[i], C.n_cells - 1));
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    const __amdgpu_buffer_rsrc_t ra = float4_rsrc(a4, n_total), rb = float4_rsrc(b4, n_total);
    walk_pairs<G, 2>(
        nbr, i, cnt, n_total, dim,
        [&](uint32_t e, float4* v) {
            v[0] = gather4(ra, e);
            v[1] = gather4(rb, e);
        },
        [&](uint32_t, const float4* v, uint32_t code) {
            const float4& aj = v[0];
            const float4& bj = v[1];
            float3 d, sg = make_float3(1.0f, 1.0f, 1.0f);
            if constexpr (kMirror) d = pair_d_img(tab.v[code], code, M, aj.x, aj.y, aj.z, ai4.x, ai4.y, ai4.z, &sg);
            else d = pair_d(tab.v[code], aj.x, aj.y, aj.z, ai4.x, ai4.y, ai4.z);
            const float vjx = kMirror ? sg.x * bj.x : bj.x;
            const float vjy = kMirror ? sg.y * bj.y : bj.y;
            const float vjz = kMirror ? sg.z * bj.z : bj.z;
            const float r2 = pair_r2(d, dim);
            const float q = pair_sqrt(r2) * inv_h;
            const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
            const float F = C.F_coef * (t * t * t);  // 0 for padding pairs (t = 0)
            if constexpr (kModel == NAUTICLE_MODEL_SUMMATION) {
                // pressure: -m (s_i + s_j) F r_ij = +m (s_i + s_j) F d
                const float cp = m * (ai4.w + aj.w) * F;
                // viscosity: m nu (k_i + k_j) F (v_i - v_j)
                const float cv = mnu * (bi4.w + bj.w) * F;
                ax = fmaf(cp, d.x, fmaf(cv, bi4.x - vjx, ax));
                ay = fmaf(cp, d.y, fmaf(cv, bi4.y - vjy, ay));
                az = fmaf(cp, d.z, fmaf(cv, bi4.z - vjz, az));
            } else {
                // w = (v_i - v_j) . r_ij = -(v_i - v_j) . d
                const float w = -fmaf(bi4.z - vjz, d.z, fmaf(bi4.y - vjy, d.y, (bi4.x - vjx) * d.x));
                const float pw = w < 0.0f ? w * __builtin_amdgcn_rcpf(r2) : 0.0f;
                // -(m (s_i + s_j) + Pi_ij m) F r_ij = F (m (s_i + s_j) - cav pw) d
                const float c = F * fmaf(-cav, pw, m * (ai4.w + aj.w));
                ax = fmaf(c, d.x, ax);
                ay = fmaf(c, d.y, ay);
                az = fmaf(c, d.z, az);
            }
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
        if constexpr (kModel == NAUTICLE_MODEL_CONTINUITY) next.rho[i] = f.rho[i];
    }
}

template <bool kIntegrate, int kModel, bool kMirror, uint32_t G>
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
            forces_particle<kIntegrate, kModel, kMirror, G>(C, tab, it.first + threadIdx.x, st, a4, b4, nbr, nbr_count,
                                                         max_nbr, n_total, f, next, err);
    });
}

using Kern = decltype(&k_forces<true, NAUTICLE_MODEL_SUMMATION, false, kGroup3>);

// The force kernel for a plan: [integrate][model][mirror] at group size G.
template <uint32_t G>
Kern forces_kernel(const Plan& P, bool integrate)
{
    static const Kern table[2][2][2] = {
        {{k_forces<false, NAUTICLE_MODEL_SUMMATION, false, G>, k_forces<false, NAUTICLE_MODEL_SUMMATION, true, G>},
         {k_forces<false, NAUTICLE_MODEL_CONTINUITY, false, G>, k_forces<false, NAUTICLE_MODEL_CONTINUITY, true, G>}},
        {{k_forces<true, NAUTICLE_MODEL_SUMMATION, false, G>, k_forces<true, NAUTICLE_MODEL_SUMMATION, true, G>},
         {k_forces<true, NAUTICLE_MODEL_CONTINUITY, false, G>, k_forces<true, NAUTICLE_MODEL_CONTINUITY, true, G>}}};
    return table[integrate ? 1 : 0][P.model == NAUTICLE_MODEL_CONTINUITY ? 1 : 0][P.mirror ? 1 : 0];
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
    const Kern kern = P.dim_max == 3 ? forces_kernel<kGroup3>(P, next != nullptr)
                                     : forces_kernel<kGroup2>(P, next != nullptr);
    const StateDev none{};
    kern<<<grid_for(P, reinterpret_cast<const void*>(kern)), P.block, 0, s>>>(cases, items, Q, sorted, pk.a4, pk.b4, cells.nbr, cells.nbr_count, mx,
                                         P.n_total, f, next ? *next : none, err);
    return hipGetLastError();
}

}  // namespace nau
