// Pair laws on the shared neighbour loop (gfx950): per-step packing of the
// records a law gathers, and the generic pass k_interact<Law, ...> that walks
// the neighbour lists (pipelined walk of pairs.h, image-aware), sums the
// law's pair forces, adds the particle's own term and g, and optionally
// completes the semi-implicit Euler step in the same kernel.  The laws
// themselves are in laws.h.
#include "internal.h"
#include "laws.h"
#include "pairs.h"

namespace nau {

// Records of sorted particle i from the caller's id-indexed attributes and
// the sorted state; radii above h (contacts beyond the stencil) set the
// attribute error bit.
template <class Law>
__global__ void __launch_bounds__(kMaxBlock)
k_pack_law(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
           LawAttrsDev at_, float4* __restrict__ r0, float4* __restrict__ r1, float4* __restrict__ r2,
           uint32_t* err)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const uint32_t id = st.id[i];
    const uint32_t g = C.offset + (id < C.n ? id : 0u);
    const bool fixed = id >= C.n_fluid;
    float o[3] = {0.0f, 0.0f, 0.0f}, v[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k)
        if (k < C.dim) {
            o[k] = st.off[k][i];
            v[k] = fixed ? 0.0f : st.vel[k][i];
        }
    const float R = at_.radius[g];
    r0[i] = make_float4(o[0], o[1], o[2], R);
    if constexpr (Law::kNA == 3) {  // DEM
        r1[i] = make_float4(v[0], v[1], v[2], at_.mass[g]);
        r2[i] = make_float4(at_.coef[g], 0.0f, 0.0f, 0.0f);
        if (!(R <= C.h) || !(R > 0.0f)) set_error(err, kErrAttribute);
    } else {  // social force
        r1[i] = make_float4(at_.coef[g], 0.0f, 0.0f, 0.0f);
        if (!(R >= 0.0f)) set_error(err, kErrAttribute);
    }
}

template <class Law, bool kIntegrate, bool kMirror, uint32_t G>
__device__ inline void interact_particle(const CaseDev& C, const ShiftTable& tab, uint32_t i, StateDev st,
                                         LawAttrsDev at_, const float4* __restrict__ r0,
                                         const float4* __restrict__ r1, const float4* __restrict__ r2,
                                         const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count,
                                         uint32_t max_nbr, uint32_t n_total, FieldsDev f, StateDev next,
                                         uint32_t* err)
{
    const int dim = C.dim;
    const float4 me = r0[i];
    const float4 m1 = r1[i];
    const float4 m2 = Law::kNA == 3 ? r2[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const typename Law::Own own = Law::own(me, m1, m2);
    uint32_t cnt = nbr_count[i];
    if (cnt > max_nbr) cnt = max_nbr;
    ImageFrame M{};
    if constexpr (kMirror) M = image_frame(C, min(st.cell[i], C.n_cells - 1));
    const __amdgpu_buffer_rsrc_t q0 = float4_rsrc(r0, n_total), q1 = float4_rsrc(r1, n_total),
                                 q2 = float4_rsrc(r2 ? r2 : r0, n_total);
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    walk_pairs<G, Law::kNA>(
        nbr, i, cnt, n_total, dim,
        [&](uint32_t e, float4* v) {
            v[0] = gather4(q0, e);
            v[1] = gather4(q1, e);
            if constexpr (Law::kNA == 3) v[2] = gather4(q2, e);
        },
        [&](uint32_t e, const float4* v, uint32_t code) {
            float3 d, sg = make_float3(1.0f, 1.0f, 1.0f);
            bool self = false;  // the particle's own mirror image (only images repeat the index)
            if constexpr (kMirror) {
                d = pair_d_img(tab.v[code], code, M, v[0].x, v[0].y, v[0].z, me.x, me.y, me.z, &sg);
                self = (e & kIndexMask) == i;
            } else {
                d = pair_d(tab.v[code], v[0].x, v[0].y, v[0].z, me.x, me.y, me.z);
            }
            const float3 F = Law::pair(C, own, v, d, pair_r2(d, dim), sg, self);
            fx += F.x;
            fy += F.y;
            fz += F.z;
        });
    const uint32_t id = st.id[i];
    const bool fixed = id >= C.n_fluid;
    const uint32_t g = C.offset + (id < C.n ? id : 0u);
    const float mass = at_.mass[g];
    const float inv_m = 1.0f / mass;
    float a[3] = {fx * inv_m, fy * inv_m, fz * inv_m};
    float vi[3] = {0.0f, 0.0f, 0.0f};
    for (int c = 0; c < 3; ++c)
        if (c < dim && !fixed) vi[c] = st.vel[c][i];
    if constexpr (Law::kNA == 2) {
        // social force: relaxation towards the desired velocity v0 e0, e0 the
        // unit vector from the (absolute FP32) position to the goal
        int32_t cc[3];
        cell_coords(C, min(st.cell[i], C.n_cells - 1), cc);
        const float oi[3] = {me.x, me.y, me.z};
        float e[3] = {0.0f, 0.0f, 0.0f};
        float e2 = 0.0f;
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) break;
            const float x = (C.origin[c] + static_cast<float>(cc[c]) * C.cs[c]) + oi[c];
            e[c] = at_.goal[c][g] - x;
            e2 = fmaf(e[c], e[c], e2);
        }
        const float inv_e = e2 > 0.0f ? 1.0f / sqrtf(e2) : 0.0f;
        const float v0 = at_.v0[g];
        for (int c = 0; c < 3; ++c)
            if (c < dim) a[c] += (v0 * e[c] * inv_e - vi[c]) / C.law[3];
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
        int32_t cc[3] = {0, 0, 0};
        cell_coords(C, st.cell[i], cc);
        const float oi[3] = {me.x, me.y, me.z};
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) break;
            const float vn = fixed ? 0.0f : fmaf(C.dt, a[c], vi[c]);
            float on = oi[c];
            int32_t cn = cc[c];
            if (!fixed) ok &= split_offset(fmaf(C.dt, vn, oi[c]), C.cs[c], C.inv_cs[c], C.nc[c], cc[c], &cn, &on);
            next.vel[c][i] = vn;
            next.off[c][i] = on;
            cc[c] = cn;
        }
        if (!ok) set_error(err, kErrOutOfDomain);
        next.cell[i] = static_cast<uint32_t>(cc[0]) +
                       static_cast<uint32_t>(C.nc[0]) *
                           (static_cast<uint32_t>(cc[1]) + static_cast<uint32_t>(C.nc[1]) * static_cast<uint32_t>(cc[2]));
        next.id[i] = id;
    }
}

// Contact lists are short (a few pairs per particle), so a wave's time is the
// latency of its gathers and more resident waves hide it: four per SIMD hold
// the DEM instances to 128 VGPRs (the stepped one with symmetric faces needs
// 129 otherwise), with no spill.
template <class Law, bool kIntegrate, bool kMirror, uint32_t G>
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_interact(const CaseDev* __restrict__ cases, const Item* __restrict__ items, ItemQueue Q, StateDev st, LawAttrsDev at_,
           const float4* __restrict__ r0, const float4* __restrict__ r1, const float4* __restrict__ r2,
           const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ nbr_count, uint32_t max_nbr,
           uint32_t n_total, FieldsDev f, StateDev next, uint32_t* err)
{
    __shared__ ShiftTable tab;
    __shared__ uint32_t s_pos;
    for_each_item(Q, &s_pos, [&](uint32_t ix) {
        const Item it = items[ix];
        const CaseDev& C = cases[it.case_id];
        fill_shift_table(C, &tab);
        if (threadIdx.x < it.count)
            interact_particle<Law, kIntegrate, kMirror, G>(C, tab, it.first + threadIdx.x, st, at_, r0, r1, r2, nbr,
                                                           nbr_count, max_nbr, n_total, f, next, err);
    });
}

// pack: write the records first (else they are in place already).
template <class Law, uint32_t G>
hipError_t launch_law(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells, LawAttrsDev at_,
                      FieldsDev f, const StateDev* next, bool pack, hipStream_t s)
{
    const Packed pk = packed(P, ws);
    float4* r0 = pk.a4;
    float4* r1 = pk.b4;
    float4* r2 = Law::kNA == 3 ? pk.adj4 : nullptr;
    const CaseDev* cases = at<CaseDev>(ws, P.L.cases);
    const Item* items = at<Item>(ws, P.L.items);
    uint32_t* err = at<uint32_t>(ws, P.L.err);
    hipError_t e = hipSuccess;
    if (pack) {
        k_pack_law<Law><<<xcd_grid(P.n_items), P.block, 0, s>>>(cases, items, P.n_items, sorted, at_, r0, r1, r2,
                                                                err);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    ItemQueue Q;
    e = item_queue(P, ws, 5, s, &Q);
    if (e != hipSuccess) return e;
    using Kern = decltype(&k_interact<Law, true, false, G>);
    static const Kern table[2][2] = {{k_interact<Law, false, false, G>, k_interact<Law, false, true, G>},
                                     {k_interact<Law, true, false, G>, k_interact<Law, true, true, G>}};
    const StateDev none{};
    const Kern kern = table[next ? 1 : 0][P.mirror ? 1 : 0];
    kern<<<grid_for(P, reinterpret_cast<const void*>(kern)), P.block, 0, s>>>(
        cases, items, Q, sorted, at_, r0, r1, r2, cells.nbr, cells.nbr_count, static_cast<uint32_t>(cells.max_nbr),
        P.n_total, f, next ? *next : none, err);
    return hipGetLastError();
}

// Contact and crowd lists are short (a handful of entries in 2-D and 3-D
// alike): groups of 4 pairs per pipeline stage, for four resident waves per
// SIMD instead of two.
constexpr uint32_t kLawGroup = 4;

hipError_t launch_interact(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                           const LawAttrsDev& attrs, FieldsDev f, const StateDev* next, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    if (P.model == NAUTICLE_MODEL_DEM)
        return launch_law<DemLaw, kLawGroup>(P, ws, sorted, cells, attrs, f, next, true, s);
    return launch_law<SocialLaw, kLawGroup>(P, ws, sorted, cells, attrs, f, next, true, s);
}

hipError_t launch_interact_on_records(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                                      const LawAttrsDev& attrs, FieldsDev f, hipStream_t s)
{
    if (P.n_items == 0 || P.model != NAUTICLE_MODEL_DEM) return hipSuccess;
    return launch_law<DemLaw, kLawGroup>(P, ws, sorted, cells, attrs, f, nullptr, false, s);
}

}  // namespace nau
