// Software-pipelined walk over a particle's neighbour list, shared by the
// density, force and adjoint passes (HIP, gfx950).  Internal header.
#pragma once

#include "internal.h"

namespace nau {

__device__ inline uint32_t entry_index(uint32_t e, uint32_t n_total)
{
    const uint32_t j = e & kIndexMask;
    return j < n_total ? j : n_total - 1;  // never out of range for lists built by the search
}

// Entries k .. k + G - 1 of particle i's list (k a multiple of G, G a
// multiple of the four-entry chunk): one 16-byte load per chunk, and the 64
// lanes of a wave read 64 adjacent chunks.  Chunks at or past the particle's
// count are not read (their entries are 0: particle 0 with no shift, one
// address for every such lane); the caller masks those pairs.
template <uint32_t G>
__device__ inline void load_entries(const uint32_t* __restrict__ nbr, uint32_t i, uint32_t k, uint32_t cnt,
                                    uint32_t n_total, uint32_t* e)
{
    static_assert(G % kChunk == 0, "groups are whole chunks");
#pragma unroll
    for (uint32_t c = 0; c < G / kChunk; ++c) {
        const uint32_t kc = k + c * kChunk;
        const uint4 v = kc < cnt ? *nbr_chunk(nbr, kc / kChunk, i, n_total) : make_uint4(0u, 0u, 0u, 0u);
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
// loads they are meant to overlap.  `gather(j, v)` fills the NA float4s of
// neighbour j; `body(k, v, code)` adds pair k (k >= cnt must be masked by
// the body) with the 6-bit cell-shift code of its entry.
template <uint32_t G, uint32_t NA>
struct PairStage {
    float4 v[G][NA];
    uint32_t code[G];
};

template <uint32_t G, uint32_t NA, typename Gather>
__device__ inline void gather_stage(const uint32_t* e, uint32_t n_total, Gather&& gather, PairStage<G, NA>& S)
{
#pragma unroll
    for (uint32_t u = 0; u < G; ++u) {
        gather(entry_index(e[u], n_total), S.v[u]);
        S.code[u] = e[u] >> NAUTICLE_NBR_INDEX_BITS;
    }
}

template <uint32_t G, uint32_t NA, typename Gather, typename Body>
__device__ inline void walk_pairs(const uint32_t* __restrict__ nbr, uint32_t i, uint32_t cnt, uint32_t n_total,
                                  Gather&& gather, Body&& body)
{
    uint32_t ex[G], ey[G];
    PairStage<G, NA> A, B;
    load_entries<G>(nbr, i, 0, cnt, n_total, ex);
    __builtin_amdgcn_sched_barrier(0);
    load_entries<G>(nbr, i, G, cnt, n_total, ey);
    __builtin_amdgcn_sched_barrier(0);
    gather_stage<G, NA>(ex, n_total, gather, A);
    __builtin_amdgcn_sched_barrier(0);
    for (uint32_t k = 0; k < cnt; k += 2 * G) {
        load_entries<G>(nbr, i, k + 2 * G, cnt, n_total, ex);
        gather_stage<G, NA>(ey, n_total, gather, B);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) body(k + u, A.v[u], A.code[u]);
        __builtin_amdgcn_sched_barrier(0);
        load_entries<G>(nbr, i, k + 3 * G, cnt, n_total, ey);
        gather_stage<G, NA>(ex, n_total, gather, A);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t u = 0; u < G; ++u) body(k + G + u, B.v[u], B.code[u]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace nau
