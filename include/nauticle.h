/*
 * nauticle.h -- C-ABI of libnauticle, the MI355X (gfx950) hot path of the
 * weakly compressible SPH step built on the Nauticle particle method
 * (B. Toth, "Nauticle: a general-purpose particle-based simulation tool",
 * arXiv:1710.08259).
 *
 * What the library computes (paper references in brackets):
 *   - every particle's neighbours: all j != i closer than the influence
 *     radius 2h, found through the cell grid of the domain [Sec. 3.2.1, "The
 *     computational domain": an axis-aligned box of cuboid cells no smaller
 *     than the influence radius; pairs farther than one cell apart ignored];
 *     optionally the lists reach a skin beyond 2h and are reused while no
 *     particle has moved far enough to enter the support unlisted (the
 *     paper reruns the search only when the layout changes [Sec. 4]);
 *   - interaction sums over those neighbours [Sec. 2.1, eq.
 *     interaction_formula]: SPH density summation with the Wendland kernel
 *     [Example 1a, kernel equation; SPH sampling expression with A = rho],
 *     a Tait equation of state (linearises to the paper's p = c^2(rho-rho0)),
 *     the symmetric pressure gradient [eq. diffop1] and Laplacian viscosity
 *     [eq. diffop3, Morris form];
 *   - the first-order semi-implicit Euler step [Example 1a, eq6 then eq7],
 *     with periodic shifting of particles that leave the box on any axis
 *     [Sec. 3.2.1];
 *   - Example 1a's own model as a second choice: the continuity equation
 *     [eq. SPH_fluid_continuity], the linear equation of state
 *     p = c^2 (rho - rho0) and the momentum equation with the artificial
 *     viscosity Pi_ij [eq. SPH_fluid_momentum], stepped as eq1..eq7;
 *   - periodic, cut-off and symmetric (mirror, free-slip) faces [Sec. 3.2.1,
 *     boundary treatments];
 *   - further pair laws on the same neighbour loop, as the paper's
 *     interaction interface allows [Sec. 6]: the DEM contact law of
 *     Example 2 [eq. DEM_force] and the social force model [eq.
 *     social_force_model];
 *   - the reverse-mode derivative of one step of the summation model (not in
 *     the paper).
 * Phases are separated like the paper's equations [Sec. 3.3: an equation is
 * finished for all particles before the next one starts]: each entry point
 * is a sequence of kernels on one stream.
 *
 * Conventions (all entry points)
 *   - All particle arrays are caller-owned DEVICE memory, structure of
 *     arrays, FP32 or uint32, indexed by a global particle index in
 *     [0, N_total), N_total = sum of the cases' n.  Case b owns
 *     [offset_b, offset_b + n_b); offsets must be increasing and contiguous
 *     (offset_0 = 0, offset_{b+1} = offset_b + n_b).
 *   - Positions are stored cell-relative: the linear index of the cell that
 *     holds the particle (x fastest: c_x + n_x (c_y + n_y c_z)) and the FP32
 *     offset from that cell's lower corner, in [0, cell_size).  The cell
 *     index absorbs the large part of the coordinate, so the offset keeps
 *     FP32 resolution of cell_size * 2^-24 anywhere in the box.
 *   - "Sorted order": after nauticle_build_cells the particles of every case
 *     are ordered by cell key (stable); global position p in sorted order
 *     belongs to the same case as input position p.
 *   - Every call validates its arguments on the host first.  A host-side
 *     error returns a negative status and enqueues nothing.  Otherwise the
 *     work is enqueued on `stream` and the call returns NAUTICLE_OK without
 *     waiting.  Conditions found by kernels (non-finite values, a neighbour
 *     list overflow, a position too far outside the box) set bits in a
 *     device error word inside the workspace; nauticle_check() reads and
 *     clears it.  No call allocates device memory; no call aborts.
 *   - The workspace `ws` (device memory, `ws_bytes` long, size from
 *     nauticle_workspace_bytes) must have been set up by nauticle_prepare()
 *     with the same case table; the library remembers, per workspace
 *     address, a fingerprint of that table and rejects a different one with
 *     NAUTICLE_ERR_WORKSPACE.  Calls that share a workspace must not run
 *     concurrently on different streams.
 *   - Limits: 2 <= dim <= 3; N_total < 2^26; total cells < 2^31;
 *     max_nbr in [1, 1024].
 */
#ifndef NAUTICLE_H
#define NAUTICLE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NAUTICLE_OK = 0,
    NAUTICLE_ERR_INVALID_ARG = -1,        /* null pointer, bad size, bad layout */
    NAUTICLE_ERR_DOMAIN = -2,             /* cell < 2h, < 3 cells on a periodic axis, ... */
    NAUTICLE_ERR_NONFINITE = -3,          /* (nauticle_check) a NaN/Inf was produced or given */
    NAUTICLE_ERR_OUT_OF_DOMAIN = -4,      /* (nauticle_check) a position beyond 2^23 cells */
    NAUTICLE_ERR_WORKSPACE = -5,          /* too small, or not prepared for these cases */
    NAUTICLE_ERR_HIP = -6,                /* a HIP runtime call failed */
    NAUTICLE_ERR_NEIGHBOUR_OVERFLOW = -7, /* (nauticle_check) a particle had > max_nbr neighbours */
    NAUTICLE_ERR_ATTRIBUTE = -8           /* (nauticle_check) a pair-law attribute out of range */
} nauticle_status;

/* Face treatments [Sec. 3.2.1].  Symmetric: a particle within 2h of the
 * face interacts with the mirror images of the particles near it (itself
 * included): positions reflected in the face, the normal velocity component
 * reversed, scalar fields unchanged. */
enum { NAUTICLE_PERIODIC = 0, NAUTICLE_CUTOFF = 1, NAUTICLE_SYMMETRIC = 2 };

/* Models of the interaction step.
 *   SUMMATION:  density summation, Tait equation of state, Morris viscosity
 *               (nu);
 *   CONTINUITY: Example 1a -- density evolved by the continuity equation,
 *               p = c0^2 (rho - rho0), artificial viscosity (alpha_av);
 *   DEM:        Example 2's contact law (nauticle_interact);
 *   SOCIAL:     the social force model (nauticle_interact);
 *   CAHN_HILLIARD: Example 1b on fixed particles (nauticle_ch_steps); its
 *               kernel is normalised in 2-D (a surface in 3-D space). */
enum {
    NAUTICLE_MODEL_SUMMATION = 0,
    NAUTICLE_MODEL_CONTINUITY = 1,
    NAUTICLE_MODEL_DEM = 2,
    NAUTICLE_MODEL_SOCIAL = 3,
    NAUTICLE_MODEL_CAHN_HILLIARD = 4
};

/* Sentinel of an empty cell in cell_start / cell_end. */
#define NAUTICLE_EMPTY 0xFFFFFFFFu

/* Neighbour-list entry: bits 0..25 hold the neighbour's global sorted
 * position, bits 26+2k..27+2k hold (cell offset along axis k) + 1, the
 * offset being the neighbour's cell minus the particle's cell, in {-1,0,1},
 * after periodic folding -- or 3 when the entry is the neighbour's mirror
 * image in a symmetric face along axis k (then the neighbour and the
 * particle share the boundary cell next to that face). */
#define NAUTICLE_NBR_INDEX_BITS 26

/* The box [Sec. 3.2.1]: ncell[k] cells of edge cell_size[k] per axis, so the
 * length is L_k = ncell[k] * cell_size[k].  cell_size is used rounded to
 * FP32; it must be >= 2h + skin (the influence radius plus the case's
 * neighbour-list skin, 0 unless set).  Periodic axes need
 * ncell >= 3, symmetric axes ncell >= 2.  Axes k >= dim must have
 * ncell[k] = 1. */
typedef struct {
    int32_t dim;
    int32_t ncell[3];
    int32_t boundary[3]; /* NAUTICLE_PERIODIC, NAUTICLE_CUTOFF or NAUTICLE_SYMMETRIC */
    double origin[3];
    double cell_size[3];
} nauticle_domain;

/* Constants of one case.  h: smoothing length (support 2h); mass: particle
 * mass m; rho0: reference density; c0: sound speed; gamma: Tait exponent
 * (B = c0^2 rho0 / gamma); nu: kinematic viscosity; dt: time step;
 * g: body acceleration; alpha_av: artificial viscosity coefficient
 * (Pi_ij = -alpha_av c0 h w / (rho_i |r_ij|^2) for approaching pairs,
 * 0.1 in Example 1a); law: constants of a pair law (DEM: law[0] = c_f, the
 * Coulomb friction coefficient; SOCIAL: law[0..3] = A, B, k, tau;
 * CAHN_HILLIARD: law[0..2] = D, gamma, the time-step factor 0.1); model:
 * NAUTICLE_MODEL_*, the same for every case of a table (SUMMATION uses gamma
 * and nu, CONTINUITY alpha_av, the pair laws law[] and per-particle
 * attributes); skin: >= 0, the neighbour lists' reach beyond the support:
 * every build (nauticle_build_cells, nauticle_step, ...) lists the pairs
 * closer than 2h + skin (FP32 predicate r^2 < fl32((2h + skin)^2), with
 * (2h + skin)^2 evaluated in FP64), so that nauticle_step_verlet can reuse
 * them; every pass's terms vanish beyond 2h, so results do not depend on
 * it (the SOCIAL model, whose force is not compactly supported, requires
 * skin = 0); reserved: 0. */
typedef struct {
    double h, mass, rho0, c0, gamma, nu, dt;
    double g[3];
    double alpha_av;
    double law[4];
    double skin;
    int32_t model;
    int32_t reserved;
} nauticle_sph_params;

/* One independent problem.  Particles whose id (position within the case
 * when binned) is >= n - n_fixed are fixed walls: they take part in every
 * sum, keep v = 0 and are not moved. */
typedef struct {
    nauticle_domain dom;
    nauticle_sph_params prm;
    int64_t offset;
    int64_t n;
    int64_t n_fixed;
} nauticle_case;

/* Particle state, cell-relative layout (see Conventions).  off[k], vel[k]
 * for k >= dim may be NULL.  id[p] is the particle's index within its case
 * at binning time; it travels with the particle through every reordering.
 * rho: the evolved density of the CONTINUITY model (required there,
 * reordered with the particles; ignored and may be NULL otherwise). */
typedef struct {
    uint32_t* cell;
    float* off[3];
    float* vel[3];
    uint32_t* id;
    float* rho;
} nauticle_state;

/* Neighbour structure, filled by nauticle_build_cells.
 *   key[p]        cell key of sorted position p (case cell base + cell);
 *   perm[p]       input position of sorted position p;
 *   cell_start/end[c]: first / one-past-last sorted position of cell key c,
 *                 NAUTICLE_EMPTY for both when the cell is empty;
 *                 length nauticle_cells_total();
 *   nbr           max_nbr * N_total entries in chunks of four, chunk-major:
 *                 entry k of sorted particle p at
 *                 nbr[4 * ((k / 4) * N_total + p) + k % 4]
 *                 (so one 16-byte load gives four consecutive entries of a
 *                 particle and the lanes of a wave read adjacent chunks);
 *                 max_nbr is a multiple of 4 and nbr is 16-byte aligned;
 *                 the entries from a particle's count to the end of its
 *                 last chunk hold a padding entry (the particle itself with
 *                 cell offset -1 on every axis of the case, whose kernel
 *                 terms are exactly zero) on which the density, force and
 *                 adjoint passes rely; entries in later chunks are
 *                 unspecified;
 *   nbr_count[p]  number of neighbours of p (the full count, even if it
 *                 exceeds max_nbr, in which case the error word is set). */
typedef struct {
    uint32_t* key;
    uint32_t* perm;
    uint32_t* cell_start;
    uint32_t* cell_end;
    uint32_t* nbr;
    uint32_t* nbr_count;
    int32_t max_nbr;
} nauticle_cells;

/* Per-particle fields in sorted order.  s = p / rho^2, inv_rho = 1 / rho.
 * drho (optional, may be NULL): drho/dt of the continuity pass. */
typedef struct {
    float* rho;
    float* p;
    float* s;
    float* inv_rho;
    float* acc[3];
    float* drho;
} nauticle_fields;

/* Launch shape of the neighbour loops (search, density, forces, adjoint),
 * chosen per workload by the autotuner; results do not depend on it.
 *   block:         particles per work item = threads per workgroup, one of
 *                  64, 128, 256 (0 = 256);
 *   persistent:    0 = one workgroup per item; 1 = a persistent grid of
 *                  groups_per_cu workgroups per compute unit pulls items
 *                  from 8 queues, one per XCD: queue x holds the items a
 *                  grid launch gives XCD x (neighbouring tiles, which share
 *                  that XCD's L2), ordered by decreasing estimated cost
 *                  (particles x expected neighbours); a workgroup empties
 *                  its own XCD's queue first, then takes from the others;
 *                  one atomic counter per queue and launch;
 *   groups_per_cu: persistent workgroups per compute unit, capped at what
 *                  the kernel's registers and LDS let be resident at once
 *                  (0 = that many). */
typedef struct {
    int32_t block;
    int32_t persistent;
    int32_t groups_per_cu;
    int32_t reserved;
} nauticle_tuning;

/* Per-particle attributes of a pair law, caller-owned device FP32 arrays
 * indexed by global particle index (case offset + id, i.e. input order at
 * binning); they travel with the particles through `id`.
 *   radius: R (DEM: R <= h, so that every contact lies within the 2h
 *           stencil, else NAUTICLE_ERR_ATTRIBUTE at nauticle_check);
 *   mass:   m;
 *   coef:   DEM: (1 - nu^2) / E (so that E' = 1 / (coef_i + coef_j));
 *           SOCIAL: the attraction c (c_ij = (c_i + c_j) / 2);
 *   v0, goal[k] (SOCIAL only; may be NULL for DEM): the desired speed and
 *           the absolute target position. */
typedef struct {
    const float* radius;
    const float* mass;
    const float* coef;
    const float* v0;
    const float* goal[3];
} nauticle_law_attrs;

/* Number of cell keys over all cases (sum of ncell products). */
int64_t nauticle_cells_total(const nauticle_case* cases, int32_t n_cases);

/* Bytes of device workspace needed for these cases (with any tuning).
 * Host only. */
nauticle_status nauticle_workspace_bytes(const nauticle_case* cases, int32_t n_cases,
                                         size_t* bytes);

/* Validates the case table on the host, writes the device case table and
 * the launch work lists into `ws`, waits for the copy to finish, and
 * records the table's fingerprint and the tuning (NULL = defaults) for
 * `ws`.  Must precede every other call on `ws`; call again whenever any
 * case constant or the tuning changes. */
nauticle_status nauticle_prepare(const nauticle_case* cases, int32_t n_cases,
                                 const nauticle_tuning* tuning, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

/* Absolute FP32 positions pos[k][i] (device, k < dim) -> cell-relative
 * state: cell, off, and id = i - offset of i's case.  Velocities are not
 * touched.  Per axis: t = fl32(x - origin); c = floor(t / cell_size) as
 * fl32(t * fl32(1/cell_size)) then corrected by one if the remainder
 * fmaf(-c, cell_size, t) falls outside [0, cell_size); the cell index then
 * wraps modulo ncell on every axis [Sec. 3.2.1 periodic shifting].
 * Positions more than 2^23 cells from the origin set OUT_OF_DOMAIN. */
nauticle_status nauticle_bin(const nauticle_case* cases, int32_t n_cases, const float* const pos[3],
                             nauticle_state* state, void* ws, size_t ws_bytes, hipStream_t stream);

/* Cell-relative state -> absolute FP32 positions (output only):
 * pos = fl32(fl32(origin + c * cell_size) + off). */
nauticle_status nauticle_unbin(const nauticle_case* cases, int32_t n_cases,
                               const nauticle_state* state, float* const pos[3], void* ws,
                               size_t ws_bytes, hipStream_t stream);

/* nauticle_unbin with every particle's position written at its global
 * input index (case offset + id) instead of its position in `state`: the
 * positions in the order of nauticle_bin's input, whatever reordering the
 * steps since have made.  pos[k] (device FP32, N_total long) is output
 * only. */
nauticle_status nauticle_unbin_by_id(const nauticle_case* cases, int32_t n_cases,
                                     const nauticle_state* state, float* const pos[3], void* ws,
                                     size_t ws_bytes, hipStream_t stream);

/* The inverse bookkeeping: out[k][p] = g[k][offset + id[p]] for every
 * particle p of `state` (only state->id is read).  Brings a per-particle
 * vector given in input order (e.g. the cotangent of the positions
 * nauticle_unbin_by_id returned) into the state's order, as
 * nauticle_sph_adjoint takes it.  g[k], out[k]: device FP32, N_total long,
 * k < dim; out must not alias g. */
nauticle_status nauticle_gather_by_id(const nauticle_case* cases, int32_t n_cases,
                                      const nauticle_state* state, const float* const g[3],
                                      float* const out[3], void* ws, size_t ws_bytes,
                                      hipStream_t stream);

/* Neighbour search [Sec. 3.2.1 cell grid]: keys, stable
 * radix sort, cell start/end table, reorder of `in` into `sorted`
 * (sorted must not alias in), then every particle's neighbour list under
 * the FP32 predicate: with delta = j's cell minus i's cell (in {-1,0,1}^dim
 * after periodic folding; no folding on cut-off axes; other pairs are never
 * neighbours), d_k = fl32(fl32(off_j,k - off_i,k) + delta_k cell_size_k) and
 * r2 = fmaf(d_z, d_z, fmaf(d_y, d_y, d_x d_x)), j is a neighbour of i iff
 * j != i and r2 < fl32(4h^2).  The pair taken the other way round gives
 * exactly -d, so j is in i's list if and only if i is in j's.
 * On a symmetric axis a stencil cell beyond the face stands for the mirror
 * image of the particle's own boundary cell: for such an axis
 * d_k = fl32(fl32(-off_j,k - off_i,k) + delta_k cell_size_k) with
 * delta_k = 0 at the lower face and 2 at the upper one, and the particle's
 * own image is a neighbour (the only case j = i).
 * Each list holds the neighbours row by row of the stencil (z offset
 * outer, y offset inner, each -1..1), and within a row in ascending sorted
 * position (the cell wrapped across a periodic x face, or the image of the
 * cell at a symmetric x face, after the others).  With the CONTINUITY
 * model, in->rho is reordered into sorted->rho. */
nauticle_status nauticle_build_cells(const nauticle_case* cases, int32_t n_cases,
                                     const nauticle_state* in, nauticle_state* sorted,
                                     nauticle_cells* cells, void* ws, size_t ws_bytes,
                                     hipStream_t stream);

/* Density and pressure of every sorted particle [SPH sampling expression
 * with A = rho; Wendland kernel]: rho_i = m alpha_D + sum_j m W(r_ij);
 * p_i = B((rho_i/rho0)^gamma - 1); also s_i = p_i/rho_i^2, inv_rho_i. */
nauticle_status nauticle_sph_density(const nauticle_case* cases, int32_t n_cases,
                                     const nauticle_state* sorted, const nauticle_cells* cells,
                                     nauticle_fields* fields, void* ws, size_t ws_bytes,
                                     hipStream_t stream);

/* Continuity pass of the CONTINUITY model [Example 1a, eq1..eq3; eq.
 * SPH_fluid_continuity, the divergence in the form of eq. diffop2]:
 *   drho_i = -rho_i sum_j (v_j - v_i) . grad_i W_ij m / rho_j
 * over the lists of nauticle_build_cells (images with reflected velocity),
 * every neighbour value taken from `sorted` (the step's start); then
 *   rho_i' = rho_i + dt drho_i,  p_i = c0^2 (rho_i' - rho0),
 * written to fields->rho, p, s = p/rho'^2, inv_rho = 1/rho' (and drho if
 * fields->drho is not NULL).  Fixed particles' velocity counts as 0; their
 * density evolves like any other.  Requires sorted->rho and the CONTINUITY
 * model. */
nauticle_status nauticle_sph_continuity(const nauticle_case* cases, int32_t n_cases,
                                        const nauticle_state* sorted, const nauticle_cells* cells,
                                        nauticle_fields* fields, void* ws, size_t ws_bytes,
                                        hipStream_t stream);

/* Accelerations [eq. diffop1 with A = p; eq. diffop3, Morris form]:
 *   a_i = -sum_j m (s_i + s_j) F_ij r_ij
 *         + sum_j m nu (inv_rho_i + inv_rho_j) F_ij (v_i - v_j) + g,
 * r_ij = r_i - r_j, F(r) = -5 alpha_D (1 - r/2h)^3 / h^2 (so that
 * grad_i W_ij = F_ij r_ij).  With the CONTINUITY model the viscous term is
 * Example 1a's artificial viscosity instead [eq. SPH_fluid_momentum]:
 *   -sum_j Pi_ij m F_ij r_ij,  Pi_ij = -alpha_av c0 h w_ij inv_rho_i / |r_ij|^2
 * when w_ij = (v_i - v_j) . r_ij < 0, else 0.  For an image neighbour v_j is
 * the reflected velocity.  Fixed particles get a = 0.  Reads rho..inv_rho
 * from `fields`, writes fields->acc.  If `next` is not NULL the step is
 * completed in the same kernel [Example 1a, eq6 then eq7]:
 * v' = v + dt a, off' = off + dt v' re-split into (cell, offset) as in
 * nauticle_bin, written to `next` in sorted order (id copied; fixed
 * particles copied unchanged; with the CONTINUITY model next->rho =
 * fields->rho).  `next` must not alias `sorted`. */
nauticle_status nauticle_sph_forces(const nauticle_case* cases, int32_t n_cases,
                                    const nauticle_state* sorted, const nauticle_cells* cells,
                                    nauticle_fields* fields, nauticle_state* next, void* ws,
                                    size_t ws_bytes, hipStream_t stream);

/* One pass of the table's pair law [Sec. 6: interaction interface] over
 * the lists of nauticle_build_cells, images included:
 *   DEM [Example 2, eq. DEM_force, effective quantities as printed]: for
 *     touching pairs (delta = R_i + R_j - |r_j - r_i| > 0), n = (r_j - r_i)/|.|,
 *     f_n = k delta^(3/2) + c delta^(1/4) (v_i - v_j).n, k = (4/3) sqrt(R') E',
 *     c = sqrt(m' k)/8; F_i += -f_n n + c_f |f_n| v_t/|v_t|,
 *     v_t = (v_j - v_i) - ((v_j - v_i).n) n, the friction only where
 *     v_t != 0 (its direction is undefined at v_t = 0) and never against the
 *     particle's own image in one symmetric face, where v_t = 0 exactly
 *     (free slip) and FP32 would leave a few ulps;
 *   SOCIAL [eq. social_force_model, pair term of its listing]: for 0 < d < 2h,
 *     F_i -= [A exp((R_ij - d)/B) + k max(R_ij - d, 0) - c_ij] n, plus the
 *     particle's own term m (v0 e0 - v)/tau, e0 towards its goal;
 * a_i = F_i / m_i + g (fixed particles: a = 0), written to fields->acc
 * (only acc is used).  If `next` is not NULL the step is completed as in
 * nauticle_sph_forces.  Requires a DEM or SOCIAL table. */
nauticle_status nauticle_interact(const nauticle_case* cases, int32_t n_cases,
                                  const nauticle_state* sorted, const nauticle_cells* cells,
                                  const nauticle_law_attrs* attrs, nauticle_fields* fields,
                                  nauticle_state* next, void* ws, size_t ws_bytes, hipStream_t stream);

/* n_steps steps of a pair law in place: build_cells(state -> workspace
 * copy), then nauticle_interact with the fused integration back into
 * `state`.  phase_events as in nauticle_step (the density slot is recorded
 * right after the neighbour lists). */
nauticle_status nauticle_step_law(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                  int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields,
                                  const nauticle_law_attrs* attrs, hipEvent_t* phase_events, void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/* n_steps of Example 1b [eq. cahnhilliard_sph_discretized; its listing's
 * eq1-eq5] on particles that do not move, so `sorted` and `cells` come
 * from one nauticle_build_cells and are reused (the paper runs the search
 * only when the layout changes [Sec. 4]).  Per step, in order:
 *   time += dt;  mu = c^3 - c - gamma L(c);  cdot = D L(mu);  c += dt cdot;
 *   dt = fac min(1 / max_i |cdot_i|, gamma / (2h)^2),
 * L(A)_i = 2 (m/rho0) sum_j (A_i - A_j) F_ij [eq. diffop3 as the example
 * discretises it], F with the kernel normalised in 2-D.  c (sorted order,
 * FP32) is updated in place; mu, cdot (optional) receive the last step's
 * fields; clock (device FP64, {time, dt} per case) is read and advanced on
 * the device, so no step waits for the host.  Requires a CAHN_HILLIARD
 * table. */
nauticle_status nauticle_ch_steps(const nauticle_case* cases, int32_t n_cases,
                                  const nauticle_state* sorted, const nauticle_cells* cells, float* c,
                                  float* mu, float* cdot, double* clock, int32_t n_steps, void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/* n_steps full steps in place: build_cells(state -> workspace copy),
 * density (SUMMATION) or continuity (CONTINUITY, state->rho evolved),
 * forces with the fused integration back into `state` (pair-law tables:
 * nauticle_step_law).  After
 * the call `state` holds the particles in the sorted order of the last
 * step; `cells` and `fields` hold that step's neighbour structure and
 * fields.  phase_events (optional, NULL or 5 * n_steps caller-created HIP
 * events) are recorded on `stream` at the start of each step, after its
 * sort and reorder, after its neighbour lists, after density and after
 * forces, for timing. */
nauticle_status nauticle_step(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                              int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields,
                              hipEvent_t* phase_events, void* ws, size_t ws_bytes, hipStream_t stream);

/* n_steps steps of the SUMMATION or CONTINUITY model as nauticle_step
 * computes them, each with its own time step from a CFL condition on the
 * sound speed and the flow speed (the paper adapts dt on the device for
 * Example 1b [its listing's eq5]; the same device-side maximum serves
 * here): before every step, per case,
 *   dt = cfl * h / (c0 + max_i |v_i|)
 * over the case's fluid particles at the step's start (|v_i| in FP32, the
 * quotient in FP64, rounded to FP32 for the step), so a case at rest takes
 * dt = cfl h / c0.  clock (device FP64, {time, dt} per case) is advanced on
 * the device: time += dt, and dt holds the last step's.  The cases' own dt
 * is ignored, and the workspace keeps it for later calls.  cfl must be
 * finite and > 0. */
nauticle_status nauticle_step_cfl(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                  int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields,
                                  double cfl, double* clock, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* One full step as nauticle_step takes it, keeping what the step's adjoint
 * (nauticle_sph_adjoint) needs: the sorted input state goes to `sorted`
 * (caller-owned, the layout of `state`) instead of a workspace copy, the
 * neighbour structure to `cells` and the fields to `fields`; `state` is
 * advanced in place.  A differentiable rollout that keeps every step's
 * record calls this once per step, so that its reverse sweep needs no
 * recomputation.  Errors as nauticle_step. */
nauticle_status nauticle_step_record(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                     nauticle_state* sorted, nauticle_cells* cells, nauticle_fields* fields,
                                     void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * hosts that forbid hipMalloc, programs that must not allocate while other
 * work on the device is being captured into a HIP graph): nauticle_step
 * with the default tuning and no caller workspace.  Its scratch is a fixed
 * array of 64 MiB in the library's device code, one per device, held from
 * the library's load until the process ends; cases needing more scratch
 * than that (nauticle_workspace_bytes; about 150 bytes per particle for a
 * 3-D table, so roughly 450,000 particles) are rejected with NAUTICLE_ERR_WORKSPACE
 * before anything is enqueued.  The call allocates nothing: it writes the
 * case table into the scratch, enqueues the steps on `stream`, then waits
 * for the stream and returns the most severe condition the kernels
 * flagged (as nauticle_check would), so no separate check call is needed.
 * Because it waits for the stream, the call itself cannot be recorded while
 * `stream` is being captured.
 * state, cells and fields as in nauticle_step (caller-owned).  Every call
 * on a device shares that device's scratch, which keeps the last call's
 * contents: calls that overlap on one device (other host threads, other
 * streams) race and must be serialised by the caller. */
nauticle_status nauticle_step_fixed_scratch(const nauticle_case* cases, int32_t n_cases,
                                            nauticle_state* state, int32_t n_steps,
                                            nauticle_cells* cells, nauticle_fields* fields,
                                            hipStream_t stream);

/* n_steps steps of the SUMMATION or CONTINUITY model, as nauticle_step
 * computes them, or of the DEM contact law, as nauticle_step_law computes
 * them (attrs as there; NULL for the SPH models), with the neighbour lists
 * reused between builds (a Verlet list).  The lists reach 2h + skin (the table's skin); a build (sort,
 * reorder, lists) runs at the first step and then only before a step at
 * whose start some particle has moved more than
 *   lim = max(skin / 2 - 2^-18 max_k cell_size_k, 0)
 * from where it was at the last build, or has left the box across a face
 * of a non-periodic axis (the build's re-split shifts it periodically, as
 * nauticle_step does in the step it leaves), so every pair closer than 2h is
 * listed at every step (two particles each within lim of their build-time
 * positions close a gap of at most 2 lim < skin; the 2^-18 cell_size margin
 * covers the FP32 rounding of the predicate and of the displacement).
 * Between builds a particle keeps its build-time cell and its offset drifts
 * (off = off + dt v may leave [0, cell_size) by up to lim), which the pair
 * arithmetic (offsets and cell differences) takes exactly; each build, and
 * the end of the call, re-split the positions into (cell, offset in
 * [0, cell_size)).  With skin = 0 every step in which a particle moves
 * rebuilds, and the result equals nauticle_step's bit for bit.
 * The decision is made on the host: after each step the library copies one
 * device word back (into a 4-byte pinned host word it allocates once per
 * host thread) and waits for that copy.  Without phase events it first
 * queues the next step's first pass (density, continuity or the contact
 * pass: they write only fields), so the device keeps working during the
 * round trip; when a build turns out to be due, that pass is redone after
 * the build.  After the call `state` holds the particles, re-split, in the
 * sorted order of the last build; `fields` hold the last step's fields and
 * `cells` the last build's lists (their cell offsets refer to the
 * build-time cells, not to `state`'s).  n_builds (optional host pointer)
 * receives the number of builds.  phase_events as in nauticle_step (in a
 * step without a build, slots 1 and 2 are recorded right after slot 0; for
 * DEM, slots 2 and 3 enclose nothing and slot 4 follows the contact pass
 * and the update).  Tables of other models are rejected with
 * NAUTICLE_ERR_INVALID_ARG. */
nauticle_status nauticle_step_verlet(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                     int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields,
                                     const nauticle_law_attrs* attrs, int32_t* n_builds,
                                     hipEvent_t* phase_events, void* ws, size_t ws_bytes, hipStream_t stream);

/* Reverse mode of one step of the SUMMATION model (the derivative the paper
 * does not have); cases with a symmetric axis or the CONTINUITY model are
 * rejected with NAUTICLE_ERR_INVALID_ARG.
 * Inputs are the step's forward quantities: `sorted` (the state the step's
 * forces pass read), `cells` (its neighbour lists and perm) and `fields`
 * (rho, p, s, inv_rho of that step).  lam_x_next / lam_v_next (device, FP32,
 * sorted order) are the cotangents of the step's output positions and
 * velocities.  Writes lam_x / lam_v, the cotangents of the step's INPUT
 * state, in the input order of the step (perm applied backwards), and ADDS
 * this step's dL/dnu and dL/dc0 to dnu[b], dc0[b] (device FP64, one per
 * case).  The neighbour set is held fixed; formulas:
 *   Vh = lam_v' + dt lam_x', A = dt Vh (fluid), A = 0 (fixed)
 *   sbar_i = -m sum_j F r_ij.(A_i - A_j); kbar_i = m nu sum_j F (v_i - v_j).(A_i - A_j)
 *   rhobar_i = sbar_i (gamma (p_i + B)/rho_i^3 - 2 p_i/rho_i^3) - kbar_i/rho_i^2
 *   lam_x_i = lam_x'_i + m sum_j F r_ij (rhobar_i + rhobar_j)
 *             - m sum_j (s_i + s_j) [F (A_i - A_j) + (F'/r) r_ij (r_ij.(A_i - A_j))]
 *             + m nu sum_j (inv_rho_i + inv_rho_j) (F'/r) r_ij ((v_i - v_j).(A_i - A_j))
 *   lam_v_i = Vh_i + m nu sum_j (inv_rho_i + inv_rho_j) F (A_i - A_j)
 *   dnu += sum_i A_i . m sum_j (inv_rho_i + inv_rho_j) F (v_i - v_j)
 *   dc0 += sum_i sbar_i (2 p_i / c0) / rho_i^2
 * Fixed particles get zero cotangents. */
nauticle_status nauticle_sph_adjoint(const nauticle_case* cases, int32_t n_cases,
                                     const nauticle_state* sorted, const nauticle_cells* cells,
                                     const nauticle_fields* fields,
                                     const float* const lam_x_next[3],
                                     const float* const lam_v_next[3], float* const lam_x[3],
                                     float* const lam_v[3], double* dnu, double* dc0, void* ws,
                                     size_t ws_bytes, hipStream_t stream);

/* Rollout loss between two states of the same cases, matched by id:
 * loss[b] = (1/(n_fluid d)) sum over fluid particles of |r_a - r_b|^2,
 * the difference taken cell-relatively with periodic folding of the cell
 * difference on periodic axes.  grad[k] (device FP32, optional) receives
 * dloss/d(position of a), in a's order.  loss (device FP64 per case) is
 * overwritten. */
nauticle_status nauticle_position_loss(const nauticle_case* cases, int32_t n_cases,
                                       const nauticle_state* a, const nauticle_state* b,
                                       double* loss, float* const grad[3], void* ws,
                                       size_t ws_bytes, hipStream_t stream);

/* Synchronises `stream`, reads and clears the device error word of `ws`,
 * and returns the most severe condition it held (NAUTICLE_OK if none). */
nauticle_status nauticle_check(void* ws, size_t ws_bytes, hipStream_t stream);

/* Message for the last non-OK status returned on this host thread. */
const char* nauticle_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NAUTICLE_H */
