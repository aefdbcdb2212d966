// Software-pipelined walk over a particle's neighbour list, shared by the
// density, force and adjoint passes (HIP, gfx950).  Internal header.
#pragma once

#include "internal.h"

namespace nau {

// The cell shift of a list entry, delta * cell_size, looked up by the entry's
// 6-bit offset code (bits 26..31) in a per-block LDS table.
struct ShiftTable {
    float4 v[64];
};

// Every thread of the block must call it (contains a barrier; the caller's
// queue loop separates successive fills by barriers).
__device__ inline void fill_shift_table(const CaseDev& C, ShiftTable* tab)
{
    for (uint32_t code = threadIdx.x; code < 64; code += blockDim.x) {
        const float sx = static_cast<float>(static_cast<int32_t>(code & 3u) - 1) * C.cs[0];
        const float sy = static_cast<float>(static_cast<int32_t>((code >> 2) & 3u) - 1) * C.cs[1];
        const float sz = static_cast<float>(static_cast<int32_t>((code >> 4) & 3u) - 1) * C.cs[2];
        tab->v[code] = make_float4(sx, sy, sz, 0.0f);
    }
    __syncthreads();
}

// r_j - r_i as the neighbour predicate forms it: the offsets are subtracted
// first and the cell shift added after, d_k = fl32(fl32(off_j,k - off_i,k) +
// shift_k), so the pair taken the other way round gives exactly -d.
__device__ inline float3 pair_d(const float4& sh, float ojx, float ojy, float ojz, float oix, float oiy, float oiz)
{
#pragma clang fp contract(off)
    return make_float3((ojx - oix) + sh.x, (ojy - oiy) + sh.y, (ojz - oiz) + sh.z);
}

// ---- symmetric faces ------------------------------------------------------------
// An entry with offset code kMirrorCode along axis k is the mirror image of
// the neighbour in a symmetric face of the particle's own boundary cell.
// Along k the particle moves by 0 cells (lower face) or 2 cells (upper
// face), which its cell decides, and the neighbour's offset and velocity
// change sign (the image's normal velocity is reversed: free slip).
struct ImageFrame {
    float shift[3];  // 0 or 2 cs per axis; read for image axes only
};

__device__ inline ImageFrame image_frame(const CaseDev& C, uint32_t cell)
{
    int32_t c[3];
    cell_coords(C, cell, c);
    ImageFrame M;
    for (int k = 0; k < 3; ++k) M.shift[k] = c[k] == 0 ? 0.0f : 2.0f * C.cs[k];
    return M;
}

// pair_d for an entry that may be an image: d_k = fl32(fl32(sg_k off_j,k -
// off_i,k) + shift_k), with sg_k = -1 and shift_k = 0 or 2 cs along image
// axes (negation is exact, so this is the search predicate's arithmetic);
// sg receives the signs for the neighbour's velocity.  Without image axes
// the values equal pair_d's.
__device__ inline float3 pair_d_img(const float4& sh, uint32_t code, const ImageFrame& M, float ojx, float ojy,
                                    float ojz, float oix, float oiy, float oiz, float3* sg)
{
#pragma clang fp contract(off)
    const bool ix = (code & 3u) == kMirrorCode;
    const bool iy = ((code >> 2) & 3u) == kMirrorCode;
    const bool iz = ((code >> 4) & 3u) == kMirrorCode;
    const float sx = ix ? -1.0f : 1.0f, sy = iy ? -1.0f : 1.0f, sz = iz ? -1.0f : 1.0f;
    *sg = make_float3(sx, sy, sz);
    return make_float3(__builtin_fmaf(sx, ojx, -oix) + (ix ? M.shift[0] : sh.x),
                       __builtin_fmaf(sy, ojy, -oiy) + (iy ? M.shift[1] : sh.y),
                       __builtin_fmaf(sz, ojz, -oiz) + (iz ? M.shift[2] : sh.z));
}

__device__ inline float pair_r2(const float3& d, int dim)
{
    float r2 = __builtin_fmaf(d.y, d.y, d.x * d.x);
    if (dim == 3) r2 = __builtin_fmaf(d.z, d.z, r2);
    return r2;
}

__device__ inline uint32_t entry_index(uint32_t e, uint32_t n_total)
{
    const uint32_t j = e & kIndexMask;
    return j < n_total ? j : n_total - 1;  // never out of range for lists built by the search
}

// Neighbour records are gathered with bounds-checked buffer loads: the byte
// offset is the entry's index times 16 (one shift), the range check is the
// buffer's own (a corrupt index reads zeros instead of faulting), so no
// clamp or 64-bit address arithmetic is spent per pair.
__device__ inline __amdgpu_buffer_rsrc_t float4_rsrc(const float4* p, uint32_t n)
{
    // word 3 0x00020000: raw dword access on CDNA
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float4*>(p), 0, static_cast<int32_t>(n * 16u), 0x00020000);
}

__device__ inline float4 gather4(__amdgpu_buffer_rsrc_t r, uint32_t e)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (e & kIndexMask) << 4, 0, 0));
}

// The same for 8-byte records (the descriptor from float2_rsrc).
__device__ inline __amdgpu_buffer_rsrc_t float2_rsrc(const float2* p, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(p), 0, static_cast<int32_t>(n * 8u), 0x00020000);
}

__device__ inline float2 gather2(__amdgpu_buffer_rsrc_t r, uint32_t e)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (e & kIndexMask) << 3, 0, 0));
}

// Entries k .. k + G - 1 of particle i's list (k a multiple of G, G a
// multiple of the four-entry chunk): one 16-byte load per chunk, and the 64
// lanes of a wave read 64 adjacent chunks.  Chunks at or past the particle's
// count are not read: they are all padding (pad_entry), so such lanes gather
// their own record again.
template <uint32_t G>
__device__ inline void load_entries(const uint32_t* __restrict__ nbr, uint32_t i, uint32_t k, uint32_t cnt,
                                    uint32_t n_total, uint32_t pad, uint32_t* e)
{
    static_assert(G % kChunk == 0, "groups are whole chunks");
#pragma unroll
    for (uint32_t c = 0; c < G / kChunk; ++c) {
        const uint32_t kc = k + c * kChunk;
        const uint4 v = kc < cnt ? *nbr_chunk(nbr, kc / kChunk, i, n_total) : make_uint4(pad, pad, pad, pad);
        e[c * kChunk + 0] = v.x;
        e[c * kChunk + 1] = v.y;
        e[c * kChunk + 2] = v.z;
        e[c * kChunk + 3] = v.w;
    }
}

// The pair loops are bound by their scattered gathers (their latency, and
// the rate at which the vector L1 serves them), not by arithmetic.
// walk_pairs runs a particle's list through a two-stage load pipeline, in
// groups of G pairs held in two register stages (A, B) that alternate
// without copies:
//
//   entries(g + 2) ; gathers(g + 1) -> B ; sum group g from A
//   entries(g + 3) ; gathers(g + 2) -> A ; sum group g + 1 from B
//
// Loads complete in issue order as far as the wait counter is concerned, so
// each group's entries are issued ahead of the gathers of the group before
// it: waiting for the entries then never waits for gathers still in flight,
// and a group is summed while the next group's gathers are outstanding.
// The scheduling barriers keep the compiler from moving the sums across the
// loads they are meant to overlap.  `gather(e, v)` fills the NA float4s of
// the neighbour of list entry e; `body(e, v, code)` adds the pair of entry e
// with the 6-bit cell-offset code of that entry.  Entries past the count (up
// to the end of the last group) are padding pairs, whose terms are exactly
// zero.  (A body that does not read e costs no register for it.)
template <uint32_t G, uint32_t NA>
struct PairStage {
    float4 v[G][NA];
    uint32_t code[G];
    uint32_t entry[G];
};

template <uint32_t G, uint32_t NA, typename Gather>
__device__ inline void gather_stage(const uint32_t* e, Gather&& gather, PairStage<G, NA>& S)
{
#pragma unroll
    for (uint32_t u = 0; u < G; ++u) {
        gather(e[u], S.v[u]);
        S.code[u] = e[u] >> NAUTICLE_NBR_INDEX_BITS;
        S.entry[u] = e[u];
    }
}

template <uint32_t G, uint32_t NA, typename Gather, typename Body>
__device__ inline void walk_pairs(const uint32_t* __restrict__ nbr, uint32_t i, uint32_t cnt, uint32_t n_total,
                                  int dim, Gather&& gather, Body&& body)
{
    const uint32_t pad = pad_entry(i, dim);
    uint32_t ex[G], ey[G];
    PairStage<G, NA> A, B;
    load_entries<G>(nbr, i, 0, cnt, n_total, pad, ex);
    __builtin_amdgcn_sched_barrier(0);
    load_entries<G>(nbr, i, G, cnt, n_total, pad, ey);
    __builtin_amdgcn_sched_barrier(0);
    gather_stage<G, NA>(ex, gather, A);
    __builtin_amdgcn_sched_barrier(0);
    for (uint32_t k = 0; k < cnt; k += 2 * G) {
        load_entries<G>(nbr, i, k + 2 * G, cnt, n_total, pad, ex);
        gather_stage<G, NA>(ey, gather, B);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) body(A.entry[u], A.v[u], A.code[u]);
        __builtin_amdgcn_sched_barrier(0);
        if (k + G >= cnt) break;  // the second half would be padding only
        load_entries<G>(nbr, i, k + 3 * G, cnt, n_total, pad, ey);
        gather_stage<G, NA>(ex, gather, A);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) body(B.entry[u], B.v[u], B.code[u]);
        __builtin_amdgcn_sched_barrier(0);
    }
}


// ---- density summation ---------------------------------------------------------
// rho_i = m alpha (1 + sum_j (1 - q/2)^4 (2q + 1)),  q = r_ij / h, summed in
// list order.
constexpr uint32_t kDensityGroup = 8;

// Square root for the pair loops: the hardware instruction (1 ulp).  The
// correctly rounded sqrtf costs a dozen more instructions per pair, and the
// pair sums are held to 1e-5 of their scale, where 1 ulp (6e-8) is invisible.
__device__ inline float pair_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Kernel term of one pair at squared distance r2 (0.5 q is exact, so
// 1 - 0.5 q rounds once however it is evaluated).
__device__ inline float density_term(float r2, float inv_h)
{
#pragma clang fp contract(off)
    const float q = pair_sqrt(r2) * inv_h;
    const float t = fmaxf(1.0f - 0.5f * q, 0.0f);
    const float t2 = t * t;
    return t2 * t2 * __builtin_fmaf(2.0f, q, 1.0f);
}

// Sum of the kernel terms of sorted particle i (offsets `me`) over its first
// cnt list entries; gather(e, v) puts the neighbour's offsets in v[0].
// kMirror: entries may be images (frame M).
// (G pairs per pipeline stage: the order of the sum does not depend on it.)
template <int DIM, bool kMirror, uint32_t G = kDensityGroup, typename Gather>
__device__ inline float density_sum(const CaseDev& C, const ShiftTable& tab, const ImageFrame& M, uint32_t i,
                                    const float4& me, const uint32_t* __restrict__ nbr, uint32_t cnt, uint32_t n_total,
                                    Gather&& gather)
{
    const float inv_h = C.inv_h;
    float sum = 0.0f;
    walk_pairs<G, 1>(nbr, i, cnt, n_total, DIM, gather, [&](uint32_t, const float4* v, uint32_t code) {
        float3 d;
        if constexpr (kMirror) {
            float3 sg;
            d = pair_d_img(tab.v[code], code, M, v[0].x, v[0].y, v[0].z, me.x, me.y, me.z, &sg);
        } else {
            d = pair_d(tab.v[code], v[0].x, v[0].y, v[0].z, me.x, me.y, me.z);
        }
        sum = __fadd_rn(sum, density_term(pair_r2(d, DIM), inv_h));  // + 0 for padding pairs
    });
    return sum;
}

// rho, the Tait pressure p = B ((rho / rho0)^gamma - 1) evaluated as
// B expm1(gamma log1p(delta)) with delta = (rho - rho0) / rho0 (no
// cancellation near rho0), s = p / rho^2 and 1 / rho of sorted particle i;
// also packs (offsets, s) and (velocity, or 0 for fixed particles, 1 / rho)
// for the force pass.
__device__ inline void density_finish(const CaseDev& C, uint32_t i, float sum, const float4& me, StateDev st,
                                      FieldsDev f, float4* __restrict__ a4, float4* __restrict__ b4, uint32_t* err)
{
    const float rho = C.m_alpha * (1.0f + sum);
    const float delta = (rho - C.rho0) * C.inv_rho0;
    const float p = C.B * expm1f(C.gamma * log1pf(delta));
    const float inv_rho = 1.0f / rho;
    const float s = p * inv_rho * inv_rho;
    f.rho[i] = rho;
    f.p[i] = p;
    f.inv_rho[i] = inv_rho;
    f.s[i] = s;
    const bool fixed = st.id[i] >= C.n_fluid;
    float v[3] = {0.0f, 0.0f, 0.0f};
    for (int c = 0; c < 3; ++c)
        if (c < C.dim && !fixed) v[c] = st.vel[c][i];
    a4[i] = make_float4(me.x, me.y, me.z, s);
    b4[i] = make_float4(v[0], v[1], v[2], inv_rho);
    if (!isfinite(rho) || !isfinite(p)) set_error(err, kErrNonFinite);
}

}  // namespace nau
