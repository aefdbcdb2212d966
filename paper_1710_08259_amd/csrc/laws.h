// Pair laws on the shared neighbour loop (HIP, gfx950).  Internal header.
//
// The paper's interaction interface (Sec. 6) separates the pairwise
// contribution from the machinery that finds the pairs and sums them.  The
// same separation, at compile time: a law is a struct with
//   kNA            float4 records gathered per neighbour (record 0 is always
//                  (offsets, radius)),
//   Own            what the particle itself needs, loaded once,
//   own(...)       loads it,
//   pair(...)      the force of one neighbour on the particle, given
//                  d = r_j - r_i (image-aware), r^2, the neighbour's records,
//                  the image's velocity signs and whether the neighbour is
//                  the particle's own mirror image.
// k_interact<Law, ...> (interact.hip) walks the lists with the pipelined
// walk of pairs.h, turns the summed force into a = F/m (+ the social force's
// own relaxation term) + g, and integrates; a new law needs a struct, its
// packing and one instantiation.
#pragma once

#include "internal.h"

namespace nau {

// Per-particle attribute arrays, indexed by global particle index (case
// offset + id), as the caller passes them.
struct LawAttrsDev {
    const float* radius;
    const float* mass;
    const float* coef;    // DEM: (1 - nu^2) / E;  social force: attraction c
    const float* v0;      // social force: desired speed
    const float* goal[3]; // social force: target position (absolute)
};

// ---- DEM contact (Example 2, eq. DEM_force) --------------------------------------
// Records: 0 = (offsets, R), 1 = (velocity, 0 for fixed particles; m),
// 2 = (q = (1 - nu^2)/E, 0, 0, 0).  For touching pairs (delta = R_i + R_j - r
// > 0), with n = d / r pointing from i to j:
//   R' = R_i R_j / (R_i + R_j), m' = m_i m_j / (m_i + m_j), E' = 1/(q_i + q_j),
//   k = (4/3) sqrt(R') E', c = sqrt(m' k) / 8,
//   f_n = k delta^(3/2) + c delta^(1/4) (v_i - v_j) . n,
//   v_t = (v_j - v_i) - ((v_j - v_i) . n) n,
//   F_i += -f_n n + c_f |f_n| v_t / |v_t|,
// the friction only where v_t != 0 (its direction is undefined at v_t = 0,
// where it is taken as 0).  Against its own image in a symmetric face a
// particle has v_t = 0 exactly (d and v_j - v_i both lie along the face
// normal), which FP32 would leave at a few ulps through the rounded normal:
// that contact has no friction.  (The image in a corner, reflected along
// two or three axes, is not normal to one face and is treated like any
// other neighbour.)
struct DemLaw {
    static constexpr uint32_t kNA = 3;
    struct Own {
        float R, m, q;
        float v[3];
    };
    __device__ static Own own(const float4& r0, const float4& r1, const float4& r2)
    {
        return Own{r0.w, r1.w, r2.x, {r1.x, r1.y, r1.z}};
    }
    __device__ static float3 pair(const CaseDev& C, const Own& o, const float4* v, const float3& d, float r2,
                                  const float3& sg, bool self)
    {
        const float r = __builtin_amdgcn_sqrtf(r2);
        const float delta = (o.R + v[0].w) - r;
        if (!(delta > 0.0f) || !(r2 > 0.0f)) return make_float3(0.0f, 0.0f, 0.0f);
        const float inv_r = 1.0f / r;
        const float nx = d.x * inv_r, ny = d.y * inv_r, nz = d.z * inv_r;
        // v_j - v_i with the image's velocity
        const float dvx = fmaf(sg.x, v[1].x, -o.v[0]);
        const float dvy = fmaf(sg.y, v[1].y, -o.v[1]);
        const float dvz = fmaf(sg.z, v[1].z, -o.v[2]);
        const float dvn = fmaf(dvz, nz, fmaf(dvy, ny, dvx * nx));
        const float Rs = o.R * v[0].w / (o.R + v[0].w);
        const float ms = o.m * v[1].w / (o.m + v[1].w);
        const float Es = 1.0f / (o.q + v[2].x);
        const float k = (4.0f / 3.0f) * __builtin_amdgcn_sqrtf(Rs) * Es;
        const float c = 0.125f * __builtin_amdgcn_sqrtf(ms * k);
        const float sd = __builtin_amdgcn_sqrtf(delta);
        const float fn = fmaf(k * delta, sd, -c * __builtin_amdgcn_sqrtf(sd) * dvn);
        const float tx = fmaf(-dvn, nx, dvx), ty = fmaf(-dvn, ny, dvy), tz = fmaf(-dvn, nz, dvz);
        const float t2 = fmaf(tz, tz, fmaf(ty, ty, tx * tx));
        // the own image reflected along exactly one axis
        const bool one_face = (sg.x < 0.0f ? 1 : 0) + (sg.y < 0.0f ? 1 : 0) + (sg.z < 0.0f ? 1 : 0) == 1;
        const float ft = t2 > 0.0f && !(self && one_face) ? C.law[0] * fabsf(fn) / __builtin_amdgcn_sqrtf(t2) : 0.0f;
        return make_float3(fmaf(ft, tx, -fn * nx), fmaf(ft, ty, -fn * ny), fmaf(ft, tz, -fn * nz));
    }
};

// ---- social force (eq. social_force_model, pair term of its listing) ------------------
// Records: 0 = (offsets, R), 1 = (c, 0, 0, 0).  For 0 < d < 2h, n = d_vec / d:
//   F_i -= [A exp((R_ij - d)/B) + k max(R_ij - d, 0) - (c_i + c_j)/2] n.
// The particle's own term (v0 e0 - v) / tau is added by the pass.
struct SocialLaw {
    static constexpr uint32_t kNA = 2;
    struct Own {
        float R, c;
    };
    __device__ static Own own(const float4& r0, const float4& r1, const float4&) { return Own{r0.w, r1.x}; }
    __device__ static float3 pair(const CaseDev& C, const Own& o, const float4* v, const float3& d, float r2,
                                  const float3&, bool)
    {
        // the list's padding pairs lie beyond 2h: only r < 2h acts
        if (!(r2 < C.R2) || !(r2 > 0.0f)) return make_float3(0.0f, 0.0f, 0.0f);
        const float r = __builtin_amdgcn_sqrtf(r2);
        const float Rij = o.R + v[0].w;
        const float gap = Rij - r;
        const float body = gap > 0.0f ? C.law[2] * gap : 0.0f;
        const float s = fmaf(C.law[0], expf(gap / C.law[1]), body) - 0.5f * (o.c + v[1].x);
        const float w = -s / r;
        return make_float3(w * d.x, w * d.y, w * d.z);
    }
};

// The DEM contact pass (accelerations only) on records that are in place
// already: packed by an earlier launch_interact on the same sorted order and
// refreshed since by the Verlet drift (steps between neighbour builds: the
// radii, masses and material constants of a sorted position do not change).
hipError_t launch_interact_on_records(const Plan& P, void* ws, StateDev sorted, const nauticle_cells& cells,
                                      const LawAttrsDev& attrs, FieldsDev f, hipStream_t s);

}  // namespace nau
