// Steps between neighbour builds (gfx950): a Verlet list on the cell-relative
// layout.
//
// The lists of a table with a skin reach 2h + skin.  Between two builds a
// particle keeps the cell it had at the build and only its offset moves, so
// the pair arithmetic d = (off_j - off_i) + delta cs (shift table, mirror
// images) stays consistent: it is linear in the offsets and its cell part is
// the build-time one.  The paper reruns the search only when the layout has
// changed (Sec. 4); a skin lets the layout change a little without a new
// search.  A particle that moved more than its case's lim (just under
// skin / 2) from its build-time position, or left the box across a face of a
// non-periodic axis, makes the next step rebuild, which first re-splits
// every offset into (cell, offset in [0, cs)) with the binning rule's own
// arithmetic (split_offset), exactly as the fused step does every step.
#include "internal.h"

namespace nau {

// Both rebuild words to 0 (start of a sequence of steps).
__global__ void k_verlet_clear(uint32_t* __restrict__ flag)
{
    if (threadIdx.x < 2) flag[threadIdx.x] = 0u;
}

// The semi-implicit Euler update of sorted particle i in place, offsets not
// re-split: v' = v + dt a, off' = off + dt v' (fixed particles: v' = 0, off
// kept), the same FP32 operations as the fused update of the force pass.
// It also refreshes what the next pair pass gathers:
// - pos4 (offsets, cell x index) for the density and continuity passes;
// - for the DEM contact law (kLaw), the motion parts of its records
//   (offsets, radius) and (velocity, mass), whose other parts stay valid
//   between builds;
// - in the continuity model, the evolved density.
// `first`: the state is the one the lists were built from, so its offsets
// become the build-time offsets off0.  A particle with |off' - off0|^2 >
// lim^2, or one that left the box across a face of a non-periodic axis
// (which the fused step shifts periodically at once, and the next build's
// re-split does the same), raises the step's rebuild word (one store per
// wave at most, and none once the word is set); workgroup 0 clears the
// other word, which the next step raises.
template <int kModel, bool kLaw>
__global__ void __launch_bounds__(kMaxBlock)
k_verlet_drift(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev st,
               FieldsDev f, float* __restrict__ off0x, float* __restrict__ off0y, float* __restrict__ off0z,
               float4* __restrict__ pos4, float4* __restrict__ rec_b, uint32_t first, uint32_t* flag_set,
               uint32_t* flag_clear, uint32_t* err)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    if (ix == 0 && threadIdx.x == 0) *flag_clear = 0u;
    const Item it = items[ix];
    bool exceed = false;
    if (threadIdx.x < it.count) {
        const CaseDev& C = cases[it.case_id];
        const uint32_t i = it.first + threadIdx.x;
        const bool fixed = st.id[i] >= C.n_fluid;
        const uint32_t cell = st.cell[i];
        int32_t cc[3];
        cell_coords(C, cell, cc);
        float* const o0[3] = {off0x, off0y, off0z};
        float o[3] = {0.0f, 0.0f, 0.0f};
        float vo[3] = {0.0f, 0.0f, 0.0f};
        float d2 = 0.0f;
        bool finite = true, left = false;
        for (int c = 0; c < 3; ++c) {
            if (c >= C.dim) break;
            const float oi = st.off[c][i];
            const float vn = fixed ? 0.0f : fmaf(C.dt, f.acc[c][i], st.vel[c][i]);
            const float on = fixed ? oi : fmaf(C.dt, vn, oi);
            const float ob = first ? oi : o0[c][i];
            if (first) o0[c][i] = oi;
            st.vel[c][i] = vn;
            st.off[c][i] = on;
            o[c] = on;
            vo[c] = vn;
            const float d = on - ob;
            d2 = fmaf(d, d, d2);
            finite &= isfinite(on);
            if (!C.periodic[c]) left |= (cc[c] == 0 && on < 0.0f) || (cc[c] == C.nc[c] - 1 && on >= C.cs[c]);
        }
        if constexpr (kLaw) {  // pos4 is the law's (offsets, radius), rec_b its (velocity, mass)
            pos4[i] = make_float4(o[0], o[1], o[2], pos4[i].w);
            rec_b[i] = make_float4(vo[0], vo[1], vo[2], rec_b[i].w);
        } else {
            pos4[i] = make_float4(o[0], o[1], o[2], static_cast<float>(cc[0]));
        }
        if constexpr (kModel == NAUTICLE_MODEL_CONTINUITY) st.rho[i] = f.rho[i];
        if (!finite) set_error(err, kErrNonFinite);
        exceed = left || d2 > C.verlet_lim2;
    }
    // one lane per wave reads the word and raises it only if still clear
    const unsigned long long vote = __ballot(exceed);
    if (vote != 0ull && (threadIdx.x & 63u) == static_cast<uint32_t>(__ffsll(vote) - 1)) {
        if (__hip_atomic_load(flag_set, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            __hip_atomic_fetch_or(flag_set, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// dst = src with the offsets re-split into (cell, offset in [0, cs)); fixed
// particles are copied as they are (they never move).
__global__ void __launch_bounds__(kMaxBlock)
k_resplit(const CaseDev* __restrict__ cases, const Item* __restrict__ items, uint32_t n_items, StateDev src,
          StateDev dst, uint32_t* err)
{
    const uint32_t ix = xcd_item(n_items);
    if (ix >= n_items) return;
    const Item it = items[ix];
    if (threadIdx.x >= it.count) return;
    const CaseDev& C = cases[it.case_id];
    const uint32_t i = it.first + threadIdx.x;
    const uint32_t id = src.id[i];
    const bool fixed = id >= C.n_fluid;
    int32_t cc[3] = {0, 0, 0};
    cell_coords(C, src.cell[i], cc);
    bool ok = true;
    for (int c = 0; c < 3; ++c) {
        if (c >= C.dim) break;
        float on = src.off[c][i];
        int32_t cn = cc[c];
        if (!fixed) ok &= split_offset(on, C.cs[c], C.inv_cs[c], C.nc[c], cc[c], &cn, &on);
        dst.off[c][i] = on;
        dst.vel[c][i] = src.vel[c][i];
        cc[c] = cn;
    }
    if (!ok) set_error(err, kErrOutOfDomain);
    dst.cell[i] = static_cast<uint32_t>(cc[0]) +
                  static_cast<uint32_t>(C.nc[0]) *
                      (static_cast<uint32_t>(cc[1]) + static_cast<uint32_t>(C.nc[1]) * static_cast<uint32_t>(cc[2]));
    dst.id[i] = id;
    if (src.rho) dst.rho[i] = src.rho[i];
}

hipError_t launch_verlet_clear(const Plan& P, void* ws, hipStream_t s)
{
    k_verlet_clear<<<1, 64, 0, s>>>(at<uint32_t>(ws, P.L.vflag));
    return hipGetLastError();
}

hipError_t launch_verlet_drift(const Plan& P, void* ws, StateDev st, FieldsDev f, bool first, int parity,
                               hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    uint32_t* flag = at<uint32_t>(ws, P.L.vflag);
    // the DEM contact pass gathers its records (a4 = (offsets, R), b4 = (v, m)), the SPH passes pos4
    const bool law = P.model == NAUTICLE_MODEL_DEM;
    const Packed pk = packed(P, ws);
    auto kern = law ? k_verlet_drift<NAUTICLE_MODEL_SUMMATION, true>
                    : (P.model == NAUTICLE_MODEL_CONTINUITY ? k_verlet_drift<NAUTICLE_MODEL_CONTINUITY, false>
                                                            : k_verlet_drift<NAUTICLE_MODEL_SUMMATION, false>);
    kern<<<xcd_grid(P.n_items), P.block, 0, s>>>(
        at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items), P.n_items, st, f, at<float>(ws, P.L.off0[0]),
        at<float>(ws, P.L.off0[1]), at<float>(ws, P.L.off0[2]), law ? pk.a4 : pk.pos4, law ? pk.b4 : nullptr,
        first ? 1u : 0u, flag + (parity & 1), flag + ((parity + 1) & 1), at<uint32_t>(ws, P.L.err));
    return hipGetLastError();
}

hipError_t launch_resplit(const Plan& P, void* ws, StateDev src, StateDev dst, hipStream_t s)
{
    if (P.n_items == 0) return hipSuccess;
    k_resplit<<<xcd_grid(P.n_items), P.block, 0, s>>>(at<CaseDev>(ws, P.L.cases), at<Item>(ws, P.L.items),
                                                      P.n_items, src, dst, at<uint32_t>(ws, P.L.err));
    return hipGetLastError();
}

}  // namespace nau
