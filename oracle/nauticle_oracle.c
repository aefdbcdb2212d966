/*
 * nauticle_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, obviously-correct CPU implementation of the weakly
 * compressible SPH step that the HIP library computes.  It exists only to
 * check that library: tests/, the package's smoke() and bench.py's
 * cpu_baseline leg may load it; nothing in paper_1710_08259_amd/ may.
 * It shares no code, header, constant or table with the HIP sources.
 *
 * Arithmetic: FP64 for every physical quantity.  The only FP32 code is the
 * part whose result is defined bit-exactly in FP32 (the binning of FP32
 * positions into cells and the FP32 neighbour predicate); it uses plain C
 * float operations and fmaf, with contraction disabled at build time
 * (-ffp-contract=off) so that every operation is rounded as written.
 *
 * Parallelism follows the paper's own scheme (Sec. "Multithreading"): the
 * particle set is split into N_t contiguous ranges of N_p/N_t particles,
 * one per thread, and a phase finishes for all particles (thread join)
 * before the next phase starts.  No particle is handled by two threads.
 *
 * Method (paper Sec. 2, "Definition of the general formulation", and
 * Sec. 5.1, Example 1):
 *   - interaction sums over all neighbours j within the influence radius
 *     (eq. interaction_formula), found through the cell grid of the domain
 *     (Sec. 3.2.1, "The computational domain": cells no smaller than the
 *     influence radius, pairs farther than one cell ignored);
 *   - Wendland kernel W = alpha_D (1 - q/2)^4 (2q + 1), q = r/h, support 2h,
 *     alpha_1 = 3/(4h), alpha_2 = 7/(4 pi h^2), alpha_3 = 21/(16 pi h^3)
 *     (Example 1a, kernel equation);
 *   - density by SPH sampling of rho itself, rho_i = sum_j m W_ij (the SPH
 *     sampling expression with A = rho, self term included);
 *   - Tait equation of state p = B((rho/rho0)^gamma - 1), B = c0^2 rho0/gamma,
 *     whose linearisation at rho0 is the paper's p = c^2 (rho - rho0);
 *   - symmetric pressure gradient (eq. diffop1 with A = p, as used in the
 *     momentum equation of Example 1a), grad_i W_ij = F(r_ij) r_ij,
 *     F(r) = (1/r) dW/dr = -5 alpha_D (1 - q/2)^3 / h^2;
 *   - Laplacian viscosity (eq. diffop3 applied to v with V_j = m/rho_j, in
 *     the Morris form nu m (1/rho_i + 1/rho_j) F_ij (v_i - v_j));
 *   - first-order semi-implicit Euler: v <- v + dt a, then r <- r + dt v
 *     with the new v (Example 1a, equations eq6 and eq7);
 *   - particles leaving the box are shifted periodically on every axis
 *     (Sec. 3.2.1);
 *   - symmetric boundaries (Sec. 3.2.1): a particle within the influence
 *     radius of a symmetric face interacts with the mirror images of the
 *     particles near that face (its own included), positions reflected in
 *     the face and the normal velocity component reversed (free slip);
 *   - the operator set of Example 1a itself: the continuity equation
 *     (eq. SPH_fluid_continuity, the divergence in the form of eq. diffop2
 *     with V_j = m/rho_j), the linear equation of state p = c^2 (rho - rho0),
 *     and the momentum equation with the artificial viscosity Pi_ij, each
 *     equation finished for all particles before the next (Sec. 3.3);
 *   - two further interaction laws on the same neighbour loop, as the
 *     paper's interaction interface allows (Sec. 6): the DEM contact law of
 *     Example 2 (eq. DEM_force with the effective quantities of eq.
 *     effective_quantities) and the social force model (eq.
 *     social_force_model, with the pair term of its listing);
 *   - Example 1b: the Cahn-Hilliard equation on a surface with the
 *     Laplacian of eq. diffop3 (sph_L0) and its adaptive time step.
 * Wall particles are ordinary particles held fixed (paper Sec. 5.3 builds
 * walls from fixed particles): they contribute density and pressure, keep
 * v = 0 and are not integrated.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_EMPTY 0xFFFFFFFFu
#define OR_MAX_THREADS 256

/* ------------------------------------------------------------------------- */
/* Problem description                                                        */
/* ------------------------------------------------------------------------- */

/* Axis-aligned box split into n[k] cells of edge cs[k]; L_k = n[k]*cs[k]. */
typedef struct {
    int32_t dim;         /* 1, 2 or 3 */
    int32_t n[3];        /* cells per axis (unused axes: 1) */
    int32_t periodic[3]; /* 1 = periodic faces */
    int32_t mirror[3];   /* 1 = symmetric faces; neither flag = cut-off */
    double origin[3];
    double cs[3];
} or_domain;

/* alpha_av: coefficient of the artificial viscosity of Example 1a,
 * Pi_ij = -alpha_av c0 h (v_ji . r_ji) / (rho_i |r_ji|^2) when approaching. */
typedef struct {
    double h, mass, rho0, c0, gamma, nu, dt;
    double g[3];
    double alpha_av;
    /* constants of the pair laws: DEM law[0] = c_f (Coulomb friction);
     * social force law[0..3] = A, B, k, tau */
    double law[4];
} or_params;

/* ------------------------------------------------------------------------- */
/* Smoothing kernel (Example 1a, Wendland kernel equation)                    */
/* ------------------------------------------------------------------------- */

double or_alpha(int32_t dim, double h)
{
    if (dim == 1) return 3.0 / (4.0 * h);
    if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
    return 21.0 / (16.0 * M_PI * h * h * h);
}

/* W(r) = alpha (1 - q/2)^4 (2q + 1) for q < 2, zero otherwise. */
double or_W(int32_t dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return or_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

/* F(r) = (1/r) dW/dr = -5 alpha (1 - q/2)^3 / h^2; finite at r = 0. */
double or_F(int32_t dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return -5.0 * or_alpha(dim, h) * t * t * t / (h * h);
}

/* dF/dr = (15 alpha / (2 h^3)) (1 - q/2)^2. */
double or_dF(int32_t dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return 7.5 * or_alpha(dim, h) * t * t / (h * h * h);
}

/* Tait equation of state. */
double or_tait(const or_params* P, double rho)
{
    double B = P->c0 * P->c0 * P->rho0 / P->gamma;
    return B * (pow(rho / P->rho0, P->gamma) - 1.0);
}

/* ------------------------------------------------------------------------- */
/* FP32 binning of positions into (cell, offset) and the FP32 neighbour       */
/* predicate.  These define the bit-exact results.                            */
/* ------------------------------------------------------------------------- */

static int64_t or_floor_mod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* Offset t (FP32, measured from the lower face of cell c along one axis) is
 * split into a whole number of cells k and a remainder in [0, cs):
 *   k = floor(t * inv_cs), off = t - k*cs (one rounding, via fmaf);
 * if rounding of t*inv_cs put k one cell off, k is corrected and off
 * recomputed; a remainder that rounds up to cs itself is pulled to the
 * largest float below cs.  The cell index then wraps modulo n (periodic
 * shifting of leaving particles, on every axis). */
static void or_split_f32(float t, float cs, float inv_cs, int64_t n, int64_t c,
                         int64_t* c_out, float* off_out)
{
    float q = t * inv_cs;
    int64_t k = (int64_t)floorf(q);
    float off = fmaf(-(float)k, cs, t);
    if (off < 0.0f) {
        k -= 1;
        off = fmaf(-(float)k, cs, t);
    } else if (off >= cs) {
        k += 1;
        off = fmaf(-(float)k, cs, t);
    }
    if (off < 0.0f) off = 0.0f;
    if (off >= cs) off = nextafterf(cs, 0.0f);
    *c_out = or_floor_mod(c + k, n);
    *off_out = off;
}

/* Absolute FP32 positions -> linear cell index (x fastest) and FP32 offsets
 * from the cell's lower corner.  pos[k] may be NULL for k >= dim. */
void or_bin_f32(const or_domain* D, int64_t n, const float* px, const float* py,
                const float* pz, uint32_t* cell, float* ox, float* oy, float* oz)
{
    const float* pos[3] = {px, py, pz};
    float* off[3] = {ox, oy, oz};
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3] = {0, 0, 0};
        for (int k = 0; k < D->dim; ++k) {
            float o = (float)D->origin[k];
            float cs = (float)D->cs[k];
            float inv = (float)(1.0 / D->cs[k]);
            float t = pos[k][i] - o;
            float r;
            or_split_f32(t, cs, inv, D->n[k], 0, &c[k], &r);
            off[k][i] = r;
        }
        cell[i] = (uint32_t)(c[0] + (int64_t)D->n[0] * (c[1] + (int64_t)D->n[1] * c[2]));
    }
}

static void or_cell_coords(const or_domain* D, uint32_t cell, int64_t c[3])
{
    int64_t v = cell;
    c[0] = v % D->n[0];
    v /= D->n[0];
    c[1] = v % D->n[1];
    c[2] = v / D->n[1];
}

/* Signed cell distance from ci to cj along axis k, folded onto the nearest
 * periodic image on periodic axes; 2 means "not adjacent". */
static int or_cell_delta(const or_domain* D, int k, int64_t ci, int64_t cj)
{
    int64_t d = cj - ci;
    int64_t n = D->n[k];
    if (D->periodic[k]) {
        if (d > n / 2) d -= n;
        if (d < -(n / 2)) d += n;
        /* n >= 3 is required, so +-1 images are distinct */
    }
    if (d < -1 || d > 1) return 2;
    return (int)d;
}

/* FP32 neighbour predicate between particle i and j whose cells differ by
 * delta (j's cell minus i's, each component in {-1,0,1}):
 *   d_k  = fl32(fl32(off_j,k - off_i,k) + delta_k * cs_k)   (delta*cs is exact)
 *   r2   = fmaf(d_z, d_z, fmaf(d_y, d_y, d_x * d_x))
 *   neighbour iff r2 < fl32(4 h^2) and j != i.
 * The offsets are subtracted first, in the frame of neither cell, and the
 * cell shift is added after.  Rounding is symmetric about zero, so the pair
 * taken the other way round gives exactly -d: the relation is symmetric, i
 * lists j if and only if j lists i, as the exact relation |r_ij| < 2h is.
 * The mirror image of j in a symmetric face of i's boundary cell (i and j
 * both in that cell) takes sign_k = -1: its coordinate along k, measured in
 * i's cell frame, is -off_j at the lower face and 2 cs - off_j at the upper
 * face, so d_k = fl32(fl32(-off_j,k - off_i,k) + delta_k cs_k) with delta_k
 * = 0 (lower) or 2 (upper).  Negation is exact, and j's image seen from i
 * is as far as i's image seen from j, so image pairs are symmetric too. */
static int or_pred_f32(const or_domain* D, float R2, const int delta[3], const int sign[3],
                       const float* offi, const float* offj)
{
    float d[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < D->dim; ++k) {
        float cs = (float)D->cs[k];
        float oj = sign[k] < 0 ? -offj[k] : offj[k];
        float diff = oj - offi[k];
        d[k] = diff + (float)delta[k] * cs;
    }
    float r2 = d[0] * d[0];
    if (D->dim >= 2) r2 = fmaf(d[1], d[1], r2);
    if (D->dim >= 3) r2 = fmaf(d[2], d[2], r2);
    return r2 < R2;
}

static float or_R2_f32(double h) { return (float)(4.0 * h * h); }

/* ------------------------------------------------------------------------- */
/* Stable counting sort by key; cell start/end table                          */
/* ------------------------------------------------------------------------- */

/* perm[p] = input position of the p-th element in key order (ties keep the
 * input order); key_sorted[p] = key[perm[p]]; start/end per key value, with
 * OR_EMPTY for both when no element has that key. */
int or_sort_keys(int64_t n, const uint32_t* key, uint32_t n_keys, uint32_t* key_sorted,
                 uint32_t* perm, uint32_t* start, uint32_t* end)
{
    int64_t* count = (int64_t*)calloc((size_t)n_keys + 1, sizeof(int64_t));
    if (!count) return -1;
    for (int64_t i = 0; i < n; ++i) count[key[i] + 1] += 1;
    for (uint32_t c = 0; c < n_keys; ++c) count[c + 1] += count[c];
    for (uint32_t c = 0; c < n_keys; ++c) {
        if (count[c + 1] > count[c]) {
            start[c] = (uint32_t)count[c];
            end[c] = (uint32_t)count[c + 1];
        } else {
            start[c] = OR_EMPTY;
            end[c] = OR_EMPTY;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t pos = count[key[i]]++;
        perm[pos] = (uint32_t)i;
        key_sorted[pos] = key[i];
    }
    free(count);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FP32 neighbour counts / lists on the (cell, offset) layout                 */
/* ------------------------------------------------------------------------- */

/* Particle list per cell, built by the stable counting sort above. */
typedef struct {
    uint32_t* start;
    uint32_t* end;
    uint32_t* perm;
    uint32_t* key_sorted;
    int64_t n_cells;
} or_cell_list;

static int or_cell_list_build(const or_domain* D, int64_t n, const uint32_t* cell, or_cell_list* L)
{
    int64_t nc = (int64_t)D->n[0] * D->n[1] * D->n[2];
    L->n_cells = nc;
    L->start = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nc);
    L->end = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nc);
    L->perm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    L->key_sorted = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    if (!L->start || !L->end || !L->perm || !L->key_sorted) return -1;
    return or_sort_keys(n, cell, (uint32_t)nc, L->key_sorted, L->perm, L->start, L->end);
}

static void or_cell_list_free(or_cell_list* L)
{
    free(L->start);
    free(L->end);
    free(L->perm);
    free(L->key_sorted);
}

/* For every particle i (or every i = which[s], s < n_eval, if which is not
 * NULL): count[s] = number of j satisfying the FP32 predicate.  If list !=
 * NULL, list[s*max_nbr + k] receives the neighbours' input indices (stencil
 * order, then index order), up to max_nbr of them, and mirror[s*max_nbr + k]
 * (if not NULL) the set of axes along which that neighbour is a mirror image
 * (bit k for axis k).  Found through the cell grid: only the 3^dim cells
 * around i's cell, where a cell beyond a symmetric face stands for the
 * mirror image of the boundary cell itself. */
int or_neighbours_f32(const or_domain* D, double h, int64_t n, const uint32_t* cell,
                      const float* ox, const float* oy, const float* oz, int64_t n_eval,
                      const int64_t* which, int32_t* count, uint32_t* list, uint8_t* mirror,
                      int32_t max_nbr)
{
    or_cell_list L;
    if (or_cell_list_build(D, n, cell, &L) != 0) return -1;
    const float* off[3] = {ox, oy, oz};
    float R2 = or_R2_f32(h);
    int span[3] = {1, 1, 1};
    for (int k = 0; k < D->dim; ++k) span[k] = 3;
    int64_t m = which ? n_eval : n;
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = which ? which[s] : s;
        int64_t ci[3];
        or_cell_coords(D, cell[i], ci);
        float offi[3] = {0, 0, 0};
        for (int k = 0; k < D->dim; ++k) offi[k] = off[k][i];
        int32_t cnt = 0;
        for (int dz = 0; dz < span[2]; ++dz)
            for (int dy = 0; dy < span[1]; ++dy)
                for (int dx = 0; dx < span[0]; ++dx) {
                    int delta[3] = {span[0] == 3 ? dx - 1 : 0, span[1] == 3 ? dy - 1 : 0,
                                    span[2] == 3 ? dz - 1 : 0};
                    int sign[3] = {1, 1, 1};
                    int64_t cj[3];
                    int ok = 1;
                    uint8_t mask = 0;
                    for (int k = 0; k < 3; ++k) {
                        int64_t c = ci[k] + delta[k];
                        if (k < D->dim) {
                            if (D->periodic[k]) {
                                c = or_floor_mod(c, D->n[k]);
                            } else if (c < 0 || c >= D->n[k]) {
                                if (!D->mirror[k]) {
                                    ok = 0;
                                } else {
                                    /* the image of i's own (boundary) cell */
                                    c = ci[k];
                                    sign[k] = -1;
                                    delta[k] = delta[k] < 0 ? 0 : 2;
                                    mask |= (uint8_t)(1u << k);
                                }
                            }
                        }
                        cj[k] = c;
                    }
                    if (!ok) continue;
                    uint32_t nc = (uint32_t)(cj[0] + (int64_t)D->n[0] * (cj[1] + (int64_t)D->n[1] * cj[2]));
                    if (L.start[nc] == OR_EMPTY) continue;
                    for (uint32_t p = L.start[nc]; p < L.end[nc]; ++p) {
                        uint32_t j = L.perm[p];
                        if ((int64_t)j == i && mask == 0) continue;
                        float offj[3] = {0, 0, 0};
                        for (int k = 0; k < D->dim; ++k) offj[k] = off[k][j];
                        if (or_pred_f32(D, R2, delta, sign, offi, offj)) {
                            if (list && cnt < max_nbr) {
                                list[s * (int64_t)max_nbr + cnt] = j;
                                if (mirror) mirror[s * (int64_t)max_nbr + cnt] = mask;
                            }
                            ++cnt;
                        }
                    }
                }
        count[s] = cnt;
    }
    or_cell_list_free(&L);
    return 0;
}

/* The same counts by brute force over all pairs and all their mirror
 * images: used to pin the cell-grid enumeration above.  Along a symmetric
 * axis the reflection in the lower face maps cell c to cell -1 - c and the
 * reflection in the upper face maps it to 2n - 1 - c; an image is a
 * candidate when its cell is adjacent to i's cell. */
void or_neighbours_f32_brute(const or_domain* D, double h, int64_t n, const uint32_t* cell,
                             const float* ox, const float* oy, const float* oz, int32_t* count)
{
    const float* off[3] = {ox, oy, oz};
    float R2 = or_R2_f32(h);
    for (int64_t i = 0; i < n; ++i) {
        int64_t ci[3];
        or_cell_coords(D, cell[i], ci);
        float offi[3] = {0, 0, 0};
        for (int k = 0; k < D->dim; ++k) offi[k] = off[k][i];
        int32_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t cj[3];
            or_cell_coords(D, cell[j], cj);
            /* image choice per axis: 0 = j itself, 1 = lower face, 2 = upper face */
            int n_img = 1;
            for (int k = 0; k < D->dim; ++k) n_img *= D->mirror[k] ? 3 : 1;
            for (int img = 0; img < n_img; ++img) {
                int delta[3] = {0, 0, 0}, sign[3] = {1, 1, 1};
                int adjacent = 1, mirrored = 0, rest = img;
                for (int k = 0; k < D->dim; ++k) {
                    int choice = 0;
                    if (D->mirror[k]) {
                        choice = rest % 3;
                        rest /= 3;
                    }
                    if (choice == 0) {
                        delta[k] = or_cell_delta(D, k, ci[k], cj[k]);
                        if (delta[k] == 2) adjacent = 0;
                    } else {
                        int64_t c_img = choice == 1 ? -1 - cj[k] : 2 * (int64_t)D->n[k] - 1 - cj[k];
                        int64_t dc = c_img - ci[k];
                        if (dc < -1 || dc > 1) adjacent = 0;
                        sign[k] = -1;
                        delta[k] = choice == 1 ? 0 : 2;
                        mirrored = 1;
                    }
                }
                if (!adjacent || (j == i && !mirrored)) continue;
                float offj[3] = {0, 0, 0};
                for (int k = 0; k < D->dim; ++k) offj[k] = off[k][j];
                cnt += or_pred_f32(D, R2, delta, sign, offi, offj);
            }
        }
        count[i] = cnt;
    }
}

/* ------------------------------------------------------------------------- */
/* FP64 neighbour search on absolute positions                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_domain* D;
    double R2;
    or_cell_list L;
    int32_t* cell_of; /* per particle cell (linear) */
} or_grid64;

static int64_t or_cell_axis64(const or_domain* D, int k, double x)
{
    int64_t c = (int64_t)floor((x - D->origin[k]) / D->cs[k]);
    if (c < 0) c = 0;
    if (c >= D->n[k]) c = D->n[k] - 1;
    return c;
}

static int or_grid64_build(or_grid64* G, const or_domain* D, double h, int64_t n, const double* x)
{
    G->D = D;
    G->R2 = 4.0 * h * h;
    uint32_t* cell = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    G->cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!cell || !G->cell_of) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3] = {0, 0, 0};
        for (int k = 0; k < D->dim; ++k) c[k] = or_cell_axis64(D, k, x[3 * i + k]);
        cell[i] = (uint32_t)(c[0] + (int64_t)D->n[0] * (c[1] + (int64_t)D->n[1] * c[2]));
        G->cell_of[i] = (int32_t)cell[i];
    }
    int rc = or_cell_list_build(D, n, cell, &G->L);
    free(cell);
    return rc;
}

static void or_grid64_free(or_grid64* G)
{
    or_cell_list_free(&G->L);
    free(G->cell_of);
}

/* r_ij = x_i - x_j, minimum image on periodic axes. */
static void or_rel(const or_domain* D, const double* xi, const double* xj, double r[3])
{
    for (int k = 0; k < 3; ++k) r[k] = 0.0;
    for (int k = 0; k < D->dim; ++k) {
        double d = xi[k] - xj[k];
        if (D->periodic[k]) {
            double L = D->n[k] * D->cs[k];
            d -= L * nearbyint(d / L);
        }
        r[k] = d;
    }
}

/* Calls visit(ctx, i, j, r_ij, |r_ij|, sgn) for every j != i with
 * |r_ij| < 2h, and for every mirror image of a particle j (i itself
 * included) in a symmetric face with |r_ij| < 2h.  For an image, r_ij is
 * measured to the reflected position (2 o_k - x_j,k in the lower face,
 * 2 (o_k + L_k) - x_j,k in the upper one) and sgn_k = -1 along each
 * reflecting axis: the image's velocity is sgn * v_j (normal component
 * reversed).  sgn is all ones for j itself.  Neighbours are enumerated from
 * the 3^dim cells around i's cell; a cell beyond a symmetric face stands for
 * the image of the boundary cell (only particles of that cell can have an
 * image within 2h of a particle in it, since cells are at least 2h wide). */
typedef void (*or_visit_fn)(void* ctx, int64_t i, int64_t j, const double r[3], double rn,
                            const double sgn[3]);

static void or_for_neighbours(const or_grid64* G, const double* x, int64_t i, or_visit_fn visit, void* ctx)
{
    const or_domain* D = G->D;
    int64_t ci[3];
    or_cell_coords(D, (uint32_t)G->cell_of[i], ci);
    int span[3] = {1, 1, 1};
    for (int k = 0; k < D->dim; ++k) span[k] = 3;
    for (int dz = 0; dz < span[2]; ++dz)
        for (int dy = 0; dy < span[1]; ++dy)
            for (int dx = 0; dx < span[0]; ++dx) {
                int delta[3] = {span[0] == 3 ? dx - 1 : 0, span[1] == 3 ? dy - 1 : 0,
                                span[2] == 3 ? dz - 1 : 0};
                int64_t cj[3];
                int ok = 1, mirrored = 0;
                /* face coordinate of the reflection along each axis (if any) */
                double face[3] = {0.0, 0.0, 0.0};
                double sgn[3] = {1.0, 1.0, 1.0};
                for (int k = 0; k < 3; ++k) {
                    int64_t c = ci[k] + delta[k];
                    if (k < D->dim) {
                        if (D->periodic[k]) {
                            c = or_floor_mod(c, D->n[k]);
                        } else if (c < 0 || c >= D->n[k]) {
                            if (!D->mirror[k]) {
                                ok = 0;
                            } else {
                                c = ci[k];
                                sgn[k] = -1.0;
                                face[k] = delta[k] < 0 ? D->origin[k] : D->origin[k] + D->n[k] * D->cs[k];
                                mirrored = 1;
                            }
                        }
                    }
                    cj[k] = c;
                }
                if (!ok) continue;
                uint32_t nc = (uint32_t)(cj[0] + (int64_t)D->n[0] * (cj[1] + (int64_t)D->n[1] * cj[2]));
                if (G->L.start[nc] == OR_EMPTY) continue;
                for (uint32_t p = G->L.start[nc]; p < G->L.end[nc]; ++p) {
                    int64_t j = G->L.perm[p];
                    if (j == i && !mirrored) continue;
                    double xj[3];
                    for (int k = 0; k < 3; ++k)
                        xj[k] = sgn[k] < 0.0 ? 2.0 * face[k] - x[3 * j + k] : x[3 * j + k];
                    double r[3];
                    or_rel(D, &x[3 * i], xj, r);
                    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                    if (r2 < G->R2) visit(ctx, i, j, r, sqrt(r2), sgn);
                }
            }
}

/* ------------------------------------------------------------------------- */
/* Thread pool in the paper's particle-decomposition style                    */
/* ------------------------------------------------------------------------- */

typedef void (*or_range_fn)(void* ctx, int64_t begin, int64_t end);

typedef struct {
    or_range_fn fn;
    void* ctx;
    int64_t begin, end;
} or_task;

static void* or_task_run(void* arg)
{
    or_task* t = (or_task*)arg;
    t->fn(t->ctx, t->begin, t->end);
    return NULL;
}

/* Runs fn over [0, n) split into nthreads contiguous ranges of about
 * n/nthreads particles; returns when every range is done. */
static void or_parallel(int64_t n, int nthreads, or_range_fn fn, void* ctx)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > OR_MAX_THREADS) nthreads = OR_MAX_THREADS;
    if (nthreads == 1 || n < 2 * nthreads) {
        fn(ctx, 0, n);
        return;
    }
    pthread_t th[OR_MAX_THREADS];
    or_task task[OR_MAX_THREADS];
    int64_t nppt = n / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        task[t].fn = fn;
        task[t].ctx = ctx;
        task[t].begin = t * nppt;
        task[t].end = (t == nthreads - 1) ? n : (t + 1) * nppt;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, or_task_run, &task[t]) != 0) break;
        ++started;
    }
    or_task_run(&task[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    for (int t = started + 1; t < nthreads; ++t) or_task_run(&task[t]);
}

/* ------------------------------------------------------------------------- */
/* Density and equation of state                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_domain* D;
    const or_params* P;
    const or_grid64* G;
    const double* x;
    const int64_t* which; /* optional subset of particles to evaluate */
    double* rho;
    double* p;
    int32_t* count;
    double acc;      /* per-visit accumulator (thread private copy) */
    int32_t cnt;
} or_density_ctx;

static void or_density_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                             const double sgn[3])
{
    (void)i; (void)j; (void)r; (void)sgn;
    or_density_ctx* ctx = (or_density_ctx*)c;
    ctx->acc += ctx->P->mass * or_W(ctx->D->dim, ctx->P->h, rn);
    ctx->cnt += 1;
}

static void or_density_range(void* c, int64_t begin, int64_t end)
{
    or_density_ctx local = *(or_density_ctx*)c;
    for (int64_t s = begin; s < end; ++s) {
        int64_t i = local.which ? local.which[s] : s;
        /* self term: W(0) = alpha */
        local.acc = local.P->mass * or_alpha(local.D->dim, local.P->h);
        local.cnt = 0;
        or_for_neighbours(local.G, local.x, i, or_density_visit, &local);
        local.rho[s] = local.acc;
        if (local.p) local.p[s] = or_tait(local.P, local.acc);
        if (local.count) local.count[s] = local.cnt;
    }
}

/* rho_i = m alpha + sum_{j != i, |r_ij| < 2h} m W(|r_ij|); p_i = Tait(rho_i).
 * x is (n,3) row-major absolute positions inside the box.  If which != NULL,
 * only particles which[0..n_eval) are evaluated, results at rho[s], p[s]. */
int or_density(const or_domain* D, const or_params* P, int64_t n, const double* x,
               int64_t n_eval, const int64_t* which, double* rho, double* p, int32_t* count,
               int nthreads)
{
    or_grid64 G;
    if (or_grid64_build(&G, D, P->h, n, x) != 0) return -1;
    or_density_ctx ctx = {D, P, &G, x, which, rho, p, count, 0.0, 0};
    or_parallel(which ? n_eval : n, nthreads, or_density_range, &ctx);
    or_grid64_free(&G);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Accelerations                                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_domain* D;
    const or_params* P;
    const or_grid64* G;
    const double* x;
    const double* v;
    const double* rho;
    const double* p;
    const uint8_t* fixed;
    const int64_t* which;
    double* a;
    double acc[3];
} or_force_ctx;

static void or_force_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                           const double sgn[3])
{
    or_force_ctx* ctx = (or_force_ctx*)c;
    const or_params* P = ctx->P;
    double F = or_F(ctx->D->dim, P->h, rn);
    double si = ctx->p[i] / (ctx->rho[i] * ctx->rho[i]);
    double sj = ctx->p[j] / (ctx->rho[j] * ctx->rho[j]);
    double visc = P->nu * (1.0 / ctx->rho[i] + 1.0 / ctx->rho[j]);
    for (int k = 0; k < 3; ++k) {
        /* symmetric pressure gradient: -m (s_i + s_j) grad_i W_ij */
        ctx->acc[k] -= P->mass * (si + sj) * F * r[k];
        /* Laplacian viscosity: m nu (1/rho_i + 1/rho_j) F_ij (v_i - v_j) */
        ctx->acc[k] += P->mass * visc * F * (ctx->v[3 * i + k] - sgn[k] * ctx->v[3 * j + k]);
    }
}

static void or_force_range(void* c, int64_t begin, int64_t end)
{
    or_force_ctx local = *(or_force_ctx*)c;
    for (int64_t s = begin; s < end; ++s) {
        int64_t i = local.which ? local.which[s] : s;
        for (int k = 0; k < 3; ++k) local.acc[k] = 0.0;
        or_for_neighbours(local.G, local.x, i, or_force_visit, &local);
        int is_fixed = local.fixed ? local.fixed[i] : 0;
        for (int k = 0; k < 3; ++k)
            local.a[3 * s + k] = is_fixed ? 0.0 : local.acc[k] + (k < local.D->dim ? local.P->g[k] : 0.0);
    }
}

/* a_i = -sum_j m (p_i/rho_i^2 + p_j/rho_j^2) F_ij r_ij
 *       + sum_j m nu (1/rho_i + 1/rho_j) F_ij (v_i - v_j) + g
 * for every non-fixed i (fixed particles get a = 0).  rho and p are inputs
 * (for all n particles); x, v, a are (n,3) row-major. */
int or_forces(const or_domain* D, const or_params* P, int64_t n, const double* x, const double* v,
              const double* rho, const double* p, const uint8_t* fixed, int64_t n_eval,
              const int64_t* which, double* a, int nthreads)
{
    or_grid64 G;
    if (or_grid64_build(&G, D, P->h, n, x) != 0) return -1;
    or_force_ctx ctx = {D, P, &G, x, v, rho, p, fixed, which, a, {0, 0, 0}};
    or_parallel(which ? n_eval : n, nthreads, or_force_range, &ctx);
    or_grid64_free(&G);
    return 0;
}


/* ------------------------------------------------------------------------- */
/* Example 1a: continuity, linear equation of state, momentum with Pi_ij      */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_domain* D;
    const or_params* P;
    const or_grid64* G;
    const double* x;
    const double* v;
    const double* rho;
    const double* p;
    const uint8_t* fixed;
    const int64_t* which;
    double* out;     /* drho (n) or a (n,3) */
    double acc[3];
} or_ex1a_ctx;

/* One term of sum_j (v_j - v_i) . grad_i W_ij m / rho_j, with grad_i W_ij =
 * F_ij r_ij and, for a mirror image, v_j reflected. */
static void or_continuity_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                                const double sgn[3])
{
    or_ex1a_ctx* ctx = (or_ex1a_ctx*)c;
    const or_params* P = ctx->P;
    double F = or_F(ctx->D->dim, P->h, rn);
    double dv_dot_grad = 0.0;
    for (int k = 0; k < 3; ++k)
        dv_dot_grad += (sgn[k] * ctx->v[3 * j + k] - ctx->v[3 * i + k]) * F * r[k];
    ctx->acc[0] += dv_dot_grad * P->mass / ctx->rho[j];
}

static void or_continuity_range(void* c, int64_t begin, int64_t end)
{
    or_ex1a_ctx local = *(or_ex1a_ctx*)c;
    for (int64_t s = begin; s < end; ++s) {
        int64_t i = local.which ? local.which[s] : s;
        local.acc[0] = 0.0;
        or_for_neighbours(local.G, local.x, i, or_continuity_visit, &local);
        local.out[s] = -local.rho[i] * local.acc[0];
    }
}

/* Continuity equation of Example 1a (eq. SPH_fluid_continuity):
 *   drho_i/dt = -rho_i sum_j (v_j - v_i) . grad_i W_ij m / rho_j
 * for every particle (fixed ones included: their density evolves too).
 * x, v are (n,3) row-major, rho (n); drho receives one value per evaluated
 * particle. */
int or_continuity(const or_domain* D, const or_params* P, int64_t n, const double* x,
                  const double* v, const double* rho, int64_t n_eval, const int64_t* which,
                  double* drho, int nthreads)
{
    or_grid64 G;
    if (or_grid64_build(&G, D, P->h, n, x) != 0) return -1;
    or_ex1a_ctx ctx = {D, P, &G, x, v, rho, NULL, NULL, which, drho, {0, 0, 0}};
    or_parallel(which ? n_eval : n, nthreads, or_continuity_range, &ctx);
    or_grid64_free(&G);
    return 0;
}

/* Linear equation of state of Example 1a: p = c^2 (rho - rho0). */
double or_linear_eos(const or_params* P, double rho)
{
    return P->c0 * P->c0 * (rho - P->rho0);
}

/* One term of the momentum equation of Example 1a:
 *   -(p_i/rho_i^2 + p_j/rho_j^2 + Pi_ij) m grad_i W_ij, with
 *   Pi_ij = -alpha_av c0 h (v_ji . r_ji) / (rho_i |r_ji|^2) if v_ji . r_ji < 0,
 *   else 0; v_ji = v_j - v_i, r_ji = r_j - r_i (so v_ji . r_ji = v_ij . r_ij).
 * A coincident pair (r = 0) has v_ji . r_ji = 0 and grad W = 0: no term. */
static void or_momentum_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                              const double sgn[3])
{
    or_ex1a_ctx* ctx = (or_ex1a_ctx*)c;
    const or_params* P = ctx->P;
    double F = or_F(ctx->D->dim, P->h, rn);
    double si = ctx->p[i] / (ctx->rho[i] * ctx->rho[i]);
    double sj = ctx->p[j] / (ctx->rho[j] * ctx->rho[j]);
    double vr = 0.0;
    for (int k = 0; k < 3; ++k) vr += (ctx->v[3 * i + k] - sgn[k] * ctx->v[3 * j + k]) * r[k];
    double Pi = vr < 0.0 ? -P->alpha_av * P->c0 * P->h * vr / (ctx->rho[i] * rn * rn) : 0.0;
    for (int k = 0; k < 3; ++k) ctx->acc[k] -= (si + sj + Pi) * P->mass * F * r[k];
}

static void or_momentum_range(void* c, int64_t begin, int64_t end)
{
    or_ex1a_ctx local = *(or_ex1a_ctx*)c;
    for (int64_t s = begin; s < end; ++s) {
        int64_t i = local.which ? local.which[s] : s;
        for (int k = 0; k < 3; ++k) local.acc[k] = 0.0;
        or_for_neighbours(local.G, local.x, i, or_momentum_visit, &local);
        int is_fixed = local.fixed ? local.fixed[i] : 0;
        for (int k = 0; k < 3; ++k)
            local.out[3 * s + k] = is_fixed ? 0.0 : local.acc[k] + (k < local.D->dim ? local.P->g[k] : 0.0);
    }
}

/* Momentum equation of Example 1a (eq. SPH_fluid_momentum):
 *   a_i = -sum_j (p_i/rho_i^2 + p_j/rho_j^2 + Pi_ij) m grad_i W_ij + g
 * for every non-fixed particle (fixed particles get a = 0).  rho and p are
 * inputs for all n particles; x, v, a are (n,3) row-major. */
int or_momentum(const or_domain* D, const or_params* P, int64_t n, const double* x,
                const double* v, const double* rho, const double* p, const uint8_t* fixed,
                int64_t n_eval, const int64_t* which, double* a, int nthreads)
{
    or_grid64 G;
    if (or_grid64_build(&G, D, P->h, n, x) != 0) return -1;
    or_ex1a_ctx ctx = {D, P, &G, x, v, rho, p, fixed, which, a, {0, 0, 0}};
    or_parallel(which ? n_eval : n, nthreads, or_momentum_range, &ctx);
    or_grid64_free(&G);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Time step                                                                  */
/* ------------------------------------------------------------------------- */

/* Periodic shifting of a coordinate into [o, o + L). */
static double or_wrap(double x, double o, double L)
{
    double y = x - L * floor((x - o) / L);
    if (y >= o + L) y = o;
    if (y < o) y = o;
    return y;
}

typedef struct {
    const or_domain* D;
    const or_params* P;
    double* x;
    double* v;
    const double* a;
    const uint8_t* fixed;
} or_integrate_ctx;

static void or_integrate_range(void* c, int64_t begin, int64_t end)
{
    or_integrate_ctx* ctx = (or_integrate_ctx*)c;
    const or_domain* D = ctx->D;
    double dt = ctx->P->dt;
    for (int64_t i = begin; i < end; ++i) {
        if (ctx->fixed && ctx->fixed[i]) continue;
        for (int k = 0; k < D->dim; ++k) {
            /* semi-implicit Euler: velocity first, then position with the new velocity */
            ctx->v[3 * i + k] += dt * ctx->a[3 * i + k];
            double L = D->n[k] * D->cs[k];
            ctx->x[3 * i + k] = or_wrap(ctx->x[3 * i + k] + dt * ctx->v[3 * i + k], D->origin[k], L);
        }
    }
}

/* Advances (x, v) by n_steps steps.  Each step recomputes neighbours,
 * density and pressure from the current positions, then accelerations, then
 * integrates.  rho, p, a (optional) receive the values of the last step. */
int or_step(const or_domain* D, const or_params* P, int64_t n, double* x, double* v,
            const uint8_t* fixed, int32_t n_steps, double* rho_out, double* p_out, double* a_out,
            int nthreads)
{
    double* rho = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* a = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!rho || !p || !a) return -1;
    int rc = 0;
    for (int32_t s = 0; s < n_steps && rc == 0; ++s) {
        rc = or_density(D, P, n, x, 0, NULL, rho, p, NULL, nthreads);
        if (rc == 0) rc = or_forces(D, P, n, x, v, rho, p, fixed, 0, NULL, a, nthreads);
        if (rc == 0) {
            or_integrate_ctx ic = {D, P, x, v, a, fixed};
            or_parallel(n, nthreads, or_integrate_range, &ic);
        }
    }
    if (rc == 0 && n_steps > 0) {
        if (rho_out) memcpy(rho_out, rho, sizeof(double) * (size_t)n);
        if (p_out) memcpy(p_out, p, sizeof(double) * (size_t)n);
        if (a_out) memcpy(a_out, a, sizeof(double) * 3 * (size_t)n);
    }
    free(rho);
    free(p);
    free(a);
    return rc;
}


/* Advances (x, v, rho) by n_steps steps of Example 1a, its equations in the
 * paper's order, each finished for all particles before the next:
 *   eq1 drho = continuity(x, v, rho);   eq2 rho <- rho + dt drho;
 *   eq3 p = c^2 (rho - rho0);           eq4/eq5 a = momentum(x, v, rho, p) + g;
 *   eq6 v <- v + dt a;                  eq7 x <- x + dt v (periodic shift).
 * Fixed particles keep x and v; their density evolves like any other.
 * drho, p, a (optional) receive the values of the last step. */
int or_step_ex1a(const or_domain* D, const or_params* P, int64_t n, double* x, double* v,
                 double* rho, const uint8_t* fixed, int32_t n_steps, double* drho_out,
                 double* p_out, double* a_out, int nthreads)
{
    size_t N = (size_t)(n > 0 ? n : 1);
    double* drho = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * N);
    double* a = (double*)malloc(sizeof(double) * 3 * N);
    if (!drho || !p || !a) return -1;
    int rc = 0;
    for (int32_t s = 0; s < n_steps && rc == 0; ++s) {
        rc = or_continuity(D, P, n, x, v, rho, 0, NULL, drho, nthreads);
        if (rc != 0) break;
        for (int64_t i = 0; i < n; ++i) {
            rho[i] += P->dt * drho[i];
            p[i] = or_linear_eos(P, rho[i]);
        }
        rc = or_momentum(D, P, n, x, v, rho, p, fixed, 0, NULL, a, nthreads);
        if (rc != 0) break;
        or_integrate_ctx ic = {D, P, x, v, a, fixed};
        or_parallel(n, nthreads, or_integrate_range, &ic);
    }
    if (rc == 0 && n_steps > 0) {
        if (drho_out) memcpy(drho_out, drho, sizeof(double) * (size_t)n);
        if (p_out) memcpy(p_out, p, sizeof(double) * (size_t)n);
        if (a_out) memcpy(a_out, a, sizeof(double) * 3 * (size_t)n);
    }
    free(drho);
    free(p);
    free(a);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Pair laws on the same neighbour loop (Sec. 6, the interaction interface)   */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_domain* D;
    const or_params* P;
    const or_grid64* G;
    const double* x;
    const double* v;
    const double* R;      /* radius */
    const double* m;      /* mass */
    const double* q;      /* DEM: (1 - nu^2) / E;  social force: c (attraction) */
    const uint8_t* fixed;
    const int64_t* which;
    double* a;
    double acc[3];
    /* conditioning of the particle's sum (test diagnostics, not physics):
     * sum of |F_ij|, and over touching contacts the smallest overlap
     * delta / (R_i + R_j) and the smallest |v_t| / |v_j - v_i| (DEM) */
    double fabs_sum, min_overlap, min_slip;
} or_law_ctx;

/* DEM contact force on i from j (Example 2, eq. DEM_force), neglecting
 * rotation.  n = (r_j - r_i) / |r_j - r_i| points from i to j; the overlap
 * is delta = R_i + R_j - |r_j - r_i|; only touching pairs (delta > 0) act.
 *   R' = R_i R_j / (R_i + R_j),  m' = m_i m_j / (m_i + m_j),
 *   E' = E_i E_j / (E_j (1 - nu_i^2) + E_i (1 - nu_j^2)) = 1 / (q_i + q_j),
 *   k = (4/3) sqrt(R') E',  c = sqrt(m' k) / 8,
 *   f_n = k delta^(3/2) + c delta^(1/4) ddelta/dt,  ddelta/dt = (v_i - v_j) . n,
 *   v_t = (v_j - v_i) - ((v_j - v_i) . n) n,  f_t = c_f |f_n| v_t / |v_t|.
 * The normal force pushes i away from j: F_i = -f_n n + f_t.  For a mirror
 * image, v_j is reflected.  r = -rel (rel = r_i - r_j as visited).
 * The friction direction v_t / |v_t| is undefined at v_t = 0, where the law
 * jumps: there the friction term is taken as 0, and it acts wherever
 * v_t != 0.  (A particle against its own image in one symmetric face has
 * v_t = 0 exactly: n and v_j - v_i both lie along the face normal, and the
 * other components of both are exact zeros.  Free slip.) */
static void or_dem_visit(void* c, int64_t i, int64_t j, const double rel[3], double rn,
                         const double sgn[3])
{
    or_law_ctx* ctx = (or_law_ctx*)c;
    double delta = ctx->R[i] + ctx->R[j] - rn;
    if (delta <= 0.0 || rn <= 0.0) return;
    double n[3], vj[3], dv[3];
    for (int k = 0; k < 3; ++k) {
        n[k] = -rel[k] / rn;
        vj[k] = sgn[k] * ctx->v[3 * j + k];
        dv[k] = vj[k] - ctx->v[3 * i + k]; /* v_j - v_i */
    }
    double Rs = ctx->R[i] * ctx->R[j] / (ctx->R[i] + ctx->R[j]);
    double ms = ctx->m[i] * ctx->m[j] / (ctx->m[i] + ctx->m[j]);
    double Es = 1.0 / (ctx->q[i] + ctx->q[j]);
    double kh = 4.0 / 3.0 * sqrt(Rs) * Es;
    double ch = sqrt(ms * kh) / 8.0;
    double dvn = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];
    double rate = -dvn; /* ddelta/dt = (v_i - v_j) . n */
    double fn = kh * pow(delta, 1.5) + ch * pow(delta, 0.25) * rate;
    double vt[3], vtn = 0.0;
    for (int k = 0; k < 3; ++k) {
        vt[k] = dv[k] - dvn * n[k];
        vtn += vt[k] * vt[k];
    }
    int slides = vtn > 0.0;
    vtn = sqrt(vtn);
    double ft = slides ? ctx->P->law[0] * fabs(fn) : 0.0;
    for (int k = 0; k < 3; ++k) {
        ctx->acc[k] += -fn * n[k];
        if (slides) ctx->acc[k] += ft * vt[k] / vtn;
    }
    ctx->fabs_sum += sqrt(fn * fn + ft * ft);
    double ov = delta / (ctx->R[i] + ctx->R[j]);
    if (ov < ctx->min_overlap) ctx->min_overlap = ov;
    double dvn2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    if (slides && dvn2 > 0.0 && vtn / sqrt(dvn2) < ctx->min_slip) ctx->min_slip = vtn / sqrt(dvn2);
}

/* Social force pair term on i from j (eq. social_force_model with the pair
 * function of its listing): with d = |r_j - r_i|, n = (r_j - r_i) / d,
 * R_ij = R_i + R_j and c_ij = (c_i + c_j) / 2,
 *   F_i -= [A exp((R_ij - d) / B) + k max(R_ij - d, 0) - c_ij] n
 * for 0 < d < 2h (the interaction radius). */
static void or_social_visit(void* c, int64_t i, int64_t j, const double rel[3], double rn,
                            const double sgn[3])
{
    (void)sgn;
    or_law_ctx* ctx = (or_law_ctx*)c;
    if (rn <= 0.0) return;
    const double* L = ctx->P->law;
    double Rij = ctx->R[i] + ctx->R[j];
    double cij = 0.5 * (ctx->q[i] + ctx->q[j]);
    double body = Rij - rn > 0.0 ? L[2] * (Rij - rn) : 0.0;
    double s = L[0] * exp((Rij - rn) / L[1]) + body - cij;
    for (int k = 0; k < 3; ++k) ctx->acc[k] -= s * (-rel[k] / rn);
    ctx->fabs_sum += fabs(s);
}

typedef struct {
    or_law_ctx base;
    int law;             /* 0 DEM, 1 social force */
    const double* v0;    /* social force: desired speed */
    const double* goal;  /* social force: (n,3) target position */
    double* diag;        /* optional (n_eval, 3): see or_law_diag */
} or_law_run;

static void or_law_range(void* c, int64_t begin, int64_t end)
{
    or_law_run* run = (or_law_run*)c;
    or_law_ctx local = run->base;
    const or_params* P = local.P;
    for (int64_t s = begin; s < end; ++s) {
        int64_t i = local.which ? local.which[s] : s;
        for (int k = 0; k < 3; ++k) local.acc[k] = 0.0;
        local.fabs_sum = 0.0;
        local.min_overlap = INFINITY;
        local.min_slip = INFINITY;
        or_for_neighbours(local.G, local.x, i, run->law == 0 ? or_dem_visit : or_social_visit, &local);
        int is_fixed = local.fixed ? local.fixed[i] : 0;
        double own[3] = {0.0, 0.0, 0.0};
        if (run->law == 1) {
            /* relaxation to the desired velocity v0 e0, e0 towards the goal */
            double e[3] = {0.0, 0.0, 0.0}, en = 0.0;
            for (int k = 0; k < local.D->dim; ++k) {
                e[k] = run->goal[3 * i + k] - local.x[3 * i + k];
                en += e[k] * e[k];
            }
            en = sqrt(en);
            for (int k = 0; k < local.D->dim; ++k) {
                double ek = en > 0.0 ? e[k] / en : 0.0;
                own[k] = (run->v0[i] * ek - local.v[3 * i + k]) / P->law[3];
            }
        }
        for (int k = 0; k < 3; ++k) {
            double ak = k < local.D->dim ? local.acc[k] / local.m[i] + own[k] + P->g[k] : 0.0;
            local.a[3 * s + k] = is_fixed ? 0.0 : ak;
        }
        if (run->diag) {
            double on = sqrt(own[0] * own[0] + own[1] * own[1] + own[2] * own[2]);
            double gn = sqrt(P->g[0] * P->g[0] + P->g[1] * P->g[1] + P->g[2] * P->g[2]);
            run->diag[3 * s + 0] = local.fabs_sum / local.m[i] + on + gn;
            run->diag[3 * s + 1] = local.min_overlap;
            run->diag[3 * s + 2] = local.min_slip;
        }
    }
}

static int or_law_d(int law, const or_domain* D, const or_params* P, int64_t n, const double* x,
                    const double* v, const double* R, const double* m, const double* q,
                    const double* v0, const double* goal, const uint8_t* fixed, int64_t n_eval,
                    const int64_t* which, double* a, double* diag, int nthreads)
{
    double Rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) Rmax = R[i] > Rmax ? R[i] : Rmax;
    /* contacts reach R_i + R_j <= 2 Rmax; the law itself cuts the rest */
    if (law == 0 && 2.0 * Rmax > 2.0 * P->h) return -5;
    or_grid64 G;
    if (or_grid64_build(&G, D, P->h, n, x) != 0) return -1;
    or_law_run run;
    memset(&run, 0, sizeof(run));
    run.base.D = D; run.base.P = P; run.base.G = &G; run.base.x = x; run.base.v = v;
    run.base.R = R; run.base.m = m; run.base.q = q; run.base.fixed = fixed; run.base.which = which;
    run.base.a = a;
    run.law = law; run.v0 = v0; run.goal = goal; run.diag = diag;
    or_parallel(which ? n_eval : n, nthreads, or_law_range, &run);
    or_grid64_free(&G);
    return 0;
}

static int or_law(int law, const or_domain* D, const or_params* P, int64_t n, const double* x,
                  const double* v, const double* R, const double* m, const double* q,
                  const double* v0, const double* goal, const uint8_t* fixed, int64_t n_eval,
                  const int64_t* which, double* a, int nthreads)
{
    return or_law_d(law, D, P, n, x, v, R, m, q, v0, goal, fixed, n_eval, which, a, NULL, nthreads);
}

/* The accelerations of a pair law (0 DEM, 1 social force) together with,
 * per evaluated particle, how well its sum is conditioned (a test
 * diagnostic, no part of the method): diag[3s] = sum_j |F_ij| / m_i + |own
 * term| + |g| (the size of the terms the acceleration is a sum of),
 * diag[3s+1] = min over touching contacts of delta / (R_i + R_j), diag[3s+2]
 * = min over sliding contacts of |v_t| / |v_j - v_i| (both +inf without
 * such contacts; DEM only). */
int or_law_diag(int law, const or_domain* D, const or_params* P, int64_t n, const double* x,
                const double* v, const double* R, const double* m, const double* q,
                const double* v0, const double* goal, const uint8_t* fixed, int64_t n_eval,
                const int64_t* which, double* a, double* diag, int nthreads)
{
    return or_law_d(law, D, P, n, x, v, R, m, q, v0, goal, fixed, n_eval, which, a, diag, nthreads);
}

/* DEM accelerations a_i = (1/m_i) sum_j F_ij + g (Example 2, eq.
 * spheres_ode_full without the tank); q_i = (1 - nu_i^2) / E_i; c_f =
 * P->law[0].  Neighbours within 2h; radii must satisfy R_i <= h. */
int or_dem(const or_domain* D, const or_params* P, int64_t n, const double* x, const double* v,
           const double* R, const double* m, const double* q, const uint8_t* fixed, int64_t n_eval,
           const int64_t* which, double* a, int nthreads)
{
    return or_law(0, D, P, n, x, v, R, m, q, NULL, NULL, fixed, n_eval, which, a, nthreads);
}

/* Social force accelerations (eq. social_force_model):
 *   a_i = (v0_i e0_i - v_i) / tau - (1/m_i) sum_j [A exp((R_ij - d)/B)
 *         + k max(R_ij - d, 0) - c_ij] n_ji + g,
 * e0_i the unit vector from r_i to goal_i; A, B, k, tau = P->law[0..3];
 * c = per-particle attraction. */
int or_social(const or_domain* D, const or_params* P, int64_t n, const double* x, const double* v,
              const double* R, const double* m, const double* c, const double* v0,
              const double* goal, const uint8_t* fixed, int64_t n_eval, const int64_t* which,
              double* a, int nthreads)
{
    return or_law(1, D, P, n, x, v, R, m, c, v0, goal, fixed, n_eval, which, a, nthreads);
}

/* n_steps semi-implicit Euler steps (eq6, eq7 of Example 1a's scheme) of
 * a pair law: law 0 DEM, 1 social force.  a (optional) receives the last
 * step's accelerations. */
int or_step_law(int law, const or_domain* D, const or_params* P, int64_t n, double* x, double* v,
                const double* R, const double* m, const double* q, const double* v0,
                const double* goal, const uint8_t* fixed, int32_t n_steps, double* a_out,
                int nthreads)
{
    double* a = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!a) return -1;
    int rc = 0;
    for (int32_t s = 0; s < n_steps && rc == 0; ++s) {
        rc = or_law(law, D, P, n, x, v, R, m, q, v0, goal, fixed, 0, NULL, a, nthreads);
        if (rc != 0) break;
        or_integrate_ctx ic = {D, P, x, v, a, fixed};
        or_parallel(n, nthreads, or_integrate_range, &ic);
    }
    if (rc == 0 && n_steps > 0 && a_out) memcpy(a_out, a, sizeof(double) * 3 * (size_t)n);
    free(a);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Example 1b: Cahn-Hilliard with the SPH Laplacian (sph_L0)                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_domain* D;
    const or_params* P;
    const or_grid64* G;
    const double* x;
    const double* A;
    const int64_t* which;
    double* out;
    int kdim;   /* dimension the kernel is normalised in */
    double acc;
} or_lap_ctx;

/* One term of eq. diffop3 as Example 1b discretises it:
 *   2 (A_j - A_i) (r_j - r_i) . grad_i W_ij / |r_j - r_i|^2 V_j
 *   = 2 (A_i - A_j) F_ij V_j      (grad_i W_ij = F_ij (r_i - r_j)),
 * V_j = m / rho0. */
static void or_lap_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                         const double sgn[3])
{
    (void)r; (void)sgn;
    or_lap_ctx* ctx = (or_lap_ctx*)c;
    double F = or_F(ctx->kdim, ctx->P->h, rn);
    ctx->acc += 2.0 * (ctx->A[i] - ctx->A[j]) * F * ctx->P->mass / ctx->P->rho0;
}

static void or_lap_range(void* c, int64_t begin, int64_t end)
{
    or_lap_ctx local = *(or_lap_ctx*)c;
    for (int64_t s = begin; s < end; ++s) {
        int64_t i = local.which ? local.which[s] : s;
        local.acc = 0.0;
        or_for_neighbours(local.G, local.x, i, or_lap_visit, &local);
        local.out[s] = local.acc;
    }
}

/* SPH Laplacian of the scalar field A (sph_L0: eq. diffop3 with V = m/rho0),
 * kernel normalised in kdim dimensions (Example 1b: 2, on a surface in 3-D
 * space). */
int or_laplacian(const or_domain* D, const or_params* P, int kdim, int64_t n, const double* x,
                 const double* A, int64_t n_eval, const int64_t* which, double* out, int nthreads)
{
    or_grid64 G;
    if (or_grid64_build(&G, D, P->h, n, x) != 0) return -1;
    or_lap_ctx ctx = {D, P, &G, x, A, which, out, kdim, 0.0};
    or_parallel(which ? n_eval : n, nthreads, or_lap_range, &ctx);
    or_grid64_free(&G);
    return 0;
}

/* n_steps of Example 1b's equations in their listed order, the particles
 * fixed (so the neighbours are found once):
 *   eq1 time += dt;  eq2 mu = c^3 - c - gamma L0(c);  eq3 cdot = D L0(mu);
 *   eq4 c += dt cdot;  eq5 dt = fac min(1 / max_i |cdot_i|, dt_g),
 * dt_g = gamma / (2h)^2; D, gamma, fac = P->law[0..2]; kernel in kdim
 * dimensions.  c is updated in place; clock = {time, dt} in/out; mu and
 * cdot (optional) receive the last step's fields. */
int or_ch_steps(const or_domain* D, const or_params* P, int kdim, int64_t n, const double* x,
                double* c, double* clock, int32_t n_steps, double* mu_out, double* cdot_out,
                int nthreads)
{
    size_t N = (size_t)(n > 0 ? n : 1);
    double* mu = (double*)malloc(sizeof(double) * N);
    double* lc = (double*)malloc(sizeof(double) * N);
    double* cdot = (double*)malloc(sizeof(double) * N);
    if (!mu || !lc || !cdot) return -1;
    double Dc = P->law[0], gamma = P->law[1], fac = P->law[2];
    double dt_g = gamma / (4.0 * P->h * P->h);
    int rc = 0;
    for (int32_t s = 0; s < n_steps && rc == 0; ++s) {
        clock[0] += clock[1];
        rc = or_laplacian(D, P, kdim, n, x, c, 0, NULL, lc, nthreads);
        if (rc != 0) break;
        for (int64_t i = 0; i < n; ++i) mu[i] = c[i] * c[i] * c[i] - c[i] - gamma * lc[i];
        rc = or_laplacian(D, P, kdim, n, x, mu, 0, NULL, cdot, nthreads);
        if (rc != 0) break;
        double mx = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            cdot[i] *= Dc;
            c[i] += clock[1] * cdot[i];
            if (fabs(cdot[i]) > mx) mx = fabs(cdot[i]);
        }
        double lim = mx > 0.0 ? 1.0 / mx : dt_g;
        clock[1] = fac * (lim < dt_g ? lim : dt_g);
    }
    if (rc == 0 && n_steps > 0) {
        if (mu_out) memcpy(mu_out, mu, sizeof(double) * (size_t)n);
        if (cdot_out) memcpy(cdot_out, cdot, sizeof(double) * (size_t)n);
    }
    free(mu);
    free(lc);
    free(cdot);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Domain validation                                                          */
/* ------------------------------------------------------------------------- */

/* 0 if the domain can be searched with a 3^dim cell stencil: every cell edge
 * at least the influence radius 2h (Sec. 3.2.1) and at least 3 cells on a
 * periodic axis (so the stencil never meets the same image twice). */
int or_validate_domain(const or_domain* D, double h)
{
    if (D->dim < 1 || D->dim > 3) return -1;
    for (int k = 0; k < D->dim; ++k) {
        if (D->n[k] < 1) return -1;
        if (D->cs[k] < 2.0 * h) return -2;
        if (D->periodic[k] && D->n[k] < 3) return -3;
        /* both faces of a symmetric axis must be distinct cells, so that a
         * boundary cell's images lie beyond one face only */
        if (D->mirror[k] && (D->periodic[k] || D->n[k] < 2)) return -3;
    }
    for (int k = D->dim; k < 3; ++k)
        if (D->n[k] != 1) return -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* One-step vector-Jacobian product (reverse mode of or_step with one step)   */
/* ------------------------------------------------------------------------- */
/*
 * Forward step, fluid particle i (fixed particles keep x and v = 0):
 *   rho_i = m alpha + m sum_j W_ij,  p_i = B((rho_i/rho0)^gamma - 1)
 *   s_i = p_i / rho_i^2,  k_i = 1 / rho_i
 *   a_i = -m sum_j (s_i + s_j) F_ij r_ij + m nu sum_j (k_i + k_j) F_ij (v_i - v_j) + g
 *   v'_i = v_i + dt a_i,  x'_i = x_i + dt v'_i
 * Given cotangents (X', V') of (x', v'), the cotangents of (x, v, nu, c0):
 *   Vh_i = V'_i + dt X'_i ;  A_i = dt Vh_i (fluid), A_i = 0 (fixed)
 *   sbar_i = -m sum_j F_ij r_ij . (A_i - A_j)
 *   kbar_i =  m nu sum_j F_ij (v_i - v_j) . (A_i - A_j)
 *   rhobar_i = sbar_i (p'(rho_i)/rho_i^2 - 2 p_i/rho_i^3) - kbar_i / rho_i^2,
 *              p'(rho) = gamma (p + B) / rho
 *   X_i = X'_i + m sum_j F_ij r_ij (rhobar_i + rhobar_j)
 *              - m sum_j (s_i + s_j) H_ij (A_i - A_j)
 *              + m nu sum_j (k_i + k_j) (F'_ij / r_ij) r_ij [(v_i - v_j) . (A_i - A_j)]
 *         with H_ij = F_ij I + (F'_ij / r_ij) r_ij r_ij^T
 *   V_i = Vh_i + m nu sum_j (k_i + k_j) F_ij (A_i - A_j)
 *   dL/dnu += sum_i A_i . m sum_j (k_i + k_j) F_ij (v_i - v_j)
 *   dL/dc0 += sum_i sbar_i (2 p_i / c0) / rho_i^2      (dp/dc0 = 2p/c0)
 * Fixed particles get X = V = 0 (their state does not depend on the
 * parameters).  The neighbour set is held fixed within the step; coincident
 * pairs (r = 0) contribute no F' term.
 */

typedef struct {
    const or_domain* D;
    const or_params* P;
    const or_grid64* G;
    const double* x;
    const double* v;
    const double* rho;
    const double* p;
    const double* A;      /* (n,3) */
    const double* rhobar; /* pass B input */
    const uint8_t* fixed;
    double* sbar;
    double* kbar;
    double* vvisc;        /* (n,3) */
    double* nubar;        /* per particle */
    double* X;            /* (n,3) pass B output (accumulated) */
    double acc_s, acc_k, acc_nu;
    double acc_v[3], acc_x[3];
} or_vjp_ctx;

static void or_vjp_a_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                           const double sgn[3])
{
    (void)sgn; /* or_step_vjp refuses domains with symmetric faces */
    or_vjp_ctx* ctx = (or_vjp_ctx*)c;
    const or_params* P = ctx->P;
    double F = or_F(ctx->D->dim, P->h, rn);
    double ki = 1.0 / ctx->rho[i], kj = 1.0 / ctx->rho[j];
    double dA[3], dv[3];
    double rdA = 0.0, vdA = 0.0;
    for (int k = 0; k < 3; ++k) {
        dA[k] = ctx->A[3 * i + k] - ctx->A[3 * j + k];
        dv[k] = ctx->v[3 * i + k] - ctx->v[3 * j + k];
        rdA += r[k] * dA[k];
        vdA += dv[k] * dA[k];
    }
    ctx->acc_s += -P->mass * F * rdA;
    ctx->acc_k += P->mass * P->nu * F * vdA;
    double w = P->mass * (ki + kj) * F;
    for (int k = 0; k < 3; ++k) ctx->acc_v[k] += P->nu * w * dA[k];
    double Ai_dv = 0.0;
    for (int k = 0; k < 3; ++k) Ai_dv += ctx->A[3 * i + k] * dv[k];
    ctx->acc_nu += w * Ai_dv;
}

static void or_vjp_a_range(void* c, int64_t begin, int64_t end)
{
    or_vjp_ctx local = *(or_vjp_ctx*)c;
    for (int64_t i = begin; i < end; ++i) {
        local.acc_s = local.acc_k = local.acc_nu = 0.0;
        for (int k = 0; k < 3; ++k) local.acc_v[k] = 0.0;
        or_for_neighbours(local.G, local.x, i, or_vjp_a_visit, &local);
        local.sbar[i] = local.acc_s;
        local.kbar[i] = local.acc_k;
        local.nubar[i] = local.acc_nu;
        for (int k = 0; k < 3; ++k) local.vvisc[3 * i + k] = local.acc_v[k];
    }
}

static void or_vjp_b_visit(void* c, int64_t i, int64_t j, const double r[3], double rn,
                           const double sgn[3])
{
    (void)sgn;
    or_vjp_ctx* ctx = (or_vjp_ctx*)c;
    const or_params* P = ctx->P;
    int dim = ctx->D->dim;
    double F = or_F(dim, P->h, rn);
    double Fp_over_r = rn > 0.0 ? or_dF(dim, P->h, rn) / rn : 0.0;
    double si = ctx->p[i] / (ctx->rho[i] * ctx->rho[i]);
    double sj = ctx->p[j] / (ctx->rho[j] * ctx->rho[j]);
    double ki = 1.0 / ctx->rho[i], kj = 1.0 / ctx->rho[j];
    double dA[3], dv[3];
    double rdA = 0.0, vdA = 0.0;
    for (int k = 0; k < 3; ++k) {
        dA[k] = ctx->A[3 * i + k] - ctx->A[3 * j + k];
        dv[k] = ctx->v[3 * i + k] - ctx->v[3 * j + k];
        rdA += r[k] * dA[k];
        vdA += dv[k] * dA[k];
    }
    double rb = ctx->rhobar[i] + ctx->rhobar[j];
    for (int k = 0; k < 3; ++k) {
        /* density geometry */
        ctx->acc_x[k] += P->mass * F * r[k] * rb;
        /* pressure Hessian: H (A_i - A_j) = F dA + (F'/r) r (r . dA) */
        ctx->acc_x[k] -= P->mass * (si + sj) * (F * dA[k] + Fp_over_r * r[k] * rdA);
        /* viscous geometry */
        ctx->acc_x[k] += P->mass * P->nu * (ki + kj) * Fp_over_r * r[k] * vdA;
    }
}

static void or_vjp_b_range(void* c, int64_t begin, int64_t end)
{
    or_vjp_ctx local = *(or_vjp_ctx*)c;
    for (int64_t i = begin; i < end; ++i) {
        for (int k = 0; k < 3; ++k) local.acc_x[k] = 0.0;
        or_for_neighbours(local.G, local.x, i, or_vjp_b_visit, &local);
        for (int k = 0; k < 3; ++k) local.X[3 * i + k] += local.acc_x[k];
    }
}

/* x, v, lam_x_next, lam_v_next, lam_x, lam_v are (n,3) row-major.  dnu and
 * dc0 receive this step's contributions (overwritten, not accumulated). */
int or_step_vjp(const or_domain* D, const or_params* P, int64_t n, const double* x,
                const double* v, const uint8_t* fixed, const double* lam_x_next,
                const double* lam_v_next, double* lam_x, double* lam_v, double* dnu,
                double* dc0, int nthreads)
{
    for (int k = 0; k < D->dim; ++k)
        if (D->mirror[k]) return -4;  /* mirror images are outside this derivative */
    size_t N = (size_t)(n > 0 ? n : 1);
    double* rho = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * N);
    double* A = (double*)malloc(sizeof(double) * 3 * N);
    double* sbar = (double*)malloc(sizeof(double) * N);
    double* kbar = (double*)malloc(sizeof(double) * N);
    double* rhobar = (double*)malloc(sizeof(double) * N);
    double* vvisc = (double*)malloc(sizeof(double) * 3 * N);
    double* nubar = (double*)malloc(sizeof(double) * N);
    if (!rho || !p || !A || !sbar || !kbar || !rhobar || !vvisc || !nubar) return -1;
    int rc = or_density(D, P, n, x, 0, NULL, rho, p, NULL, nthreads);
    or_grid64 G;
    if (rc == 0) rc = or_grid64_build(&G, D, P->h, n, x);
    if (rc != 0) return rc;

    double dt = P->dt;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            double vh = lam_v_next[3 * i + k] + dt * lam_x_next[3 * i + k];
            int fluid = !(fixed && fixed[i]) && k < D->dim;
            A[3 * i + k] = fluid ? dt * vh : 0.0;
            lam_v[3 * i + k] = fluid ? vh : 0.0;
            lam_x[3 * i + k] = fluid ? lam_x_next[3 * i + k] : 0.0;
        }

    or_vjp_ctx ctx;
    memset(&ctx, 0, sizeof(ctx));
    ctx.D = D; ctx.P = P; ctx.G = &G; ctx.x = x; ctx.v = v; ctx.rho = rho; ctx.p = p;
    ctx.A = A; ctx.rhobar = rhobar; ctx.fixed = fixed; ctx.sbar = sbar; ctx.kbar = kbar;
    ctx.vvisc = vvisc; ctx.nubar = nubar; ctx.X = lam_x;
    or_parallel(n, nthreads, or_vjp_a_range, &ctx);

    double B = P->c0 * P->c0 * P->rho0 / P->gamma;
    double sum_nu = 0.0, sum_c0 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = rho[i];
        double dp = P->gamma * (p[i] + B) / r;
        rhobar[i] = sbar[i] * (dp / (r * r) - 2.0 * p[i] / (r * r * r)) - kbar[i] / (r * r);
        sum_c0 += sbar[i] * (2.0 * p[i] / P->c0) / (r * r);
        sum_nu += nubar[i];
    }
    or_parallel(n, nthreads, or_vjp_b_range, &ctx);
    for (int64_t i = 0; i < n; ++i) {
        int fluid = !(fixed && fixed[i]);
        for (int k = 0; k < 3; ++k) {
            if (!fluid || k >= D->dim) {
                lam_x[3 * i + k] = 0.0;
                lam_v[3 * i + k] = 0.0;
            } else {
                lam_v[3 * i + k] += vvisc[3 * i + k];
            }
        }
    }
    *dnu = sum_nu;
    *dc0 = sum_c0;
    or_grid64_free(&G);
    free(rho); free(p); free(A); free(sbar); free(kbar); free(rhobar); free(vvisc); free(nubar);
    return 0;
}
