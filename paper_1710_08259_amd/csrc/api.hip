// C-ABI entry points of libnauticle: host-side validation, the per-workspace
// plan (case table fingerprint, workspace layout, particle-block work lists), and the
// launch sequences of the five phases.  See include/nauticle.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "laws.h"
#include "sort.h"

using namespace nau;

namespace {

thread_local std::string g_last_error;

nauticle_status fail(nauticle_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

nauticle_status hip_fail(hipError_t e, const char* what)
{
    return fail(NAUTICLE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint64_t fingerprint(const nauticle_case* cases, int32_t n_cases)
{
    // FNV-1a over the raw case table
    uint64_t h = 1469598103934665603ull;
    const unsigned char* p = reinterpret_cast<const unsigned char*>(cases);
    const size_t len = sizeof(nauticle_case) * static_cast<size_t>(n_cases);
    for (size_t i = 0; i < len; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h ^ static_cast<uint64_t>(n_cases);
}

struct Derived {
    Plan plan;
    std::vector<CaseDev> cases;
    std::vector<Item> items;
    std::vector<uint32_t> queue;
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validates the case table and tuning and derives the device table, the
// work list (blocks of tuning.block particles), the cost-ordered queue and
// the workspace layout.  The layout is sized for the smallest block, so one
// workspace size serves every tuning.
nauticle_status derive(const nauticle_case* cases, int32_t n_cases, const nauticle_tuning* tuning, Derived* D)
{
    nauticle_tuning tn{256, 0, 4, 0};
    if (tuning) {
        tn = *tuning;
        if (tn.block == 0) tn.block = 256;
        if ((tn.block != 64 && tn.block != 128 && tn.block != 256) || (tn.persistent != 0 && tn.persistent != 1) ||
            tn.groups_per_cu < 0 || tn.groups_per_cu > 64)
            return fail(NAUTICLE_ERR_INVALID_ARG, "tuning: block in {64,128,256}, persistent in {0,1}, groups_per_cu in [0,64]");
    }
    const int64_t block = tn.block;
    if (!cases || n_cases < 1) return fail(NAUTICLE_ERR_INVALID_ARG, "cases is null or n_cases < 1");
    D->cases.clear();
    D->items.clear();
    D->queue.clear();
    Plan& P = D->plan;
    std::memset(&P, 0, sizeof(P));
    P.n_cases = n_cases;
    const int dim0 = cases[0].dom.dim;
    const int32_t model0 = cases[0].prm.model;
    bool any_mirror = false;
    uint64_t n_total = 0, n_cells_total = 0, n_fluid_total = 0;
    int64_t worst_items = 0;
    double halo_need = 0.0;
    std::vector<double> nbr_per_particle;
    for (int32_t b = 0; b < n_cases; ++b) {
        const nauticle_case& c = cases[b];
        const nauticle_domain& d = c.dom;
        const nauticle_sph_params& q = c.prm;
        if (d.dim < 2 || d.dim > 3) return fail(NAUTICLE_ERR_DOMAIN, "case %d: dim must be 2 or 3", b);
        if (d.dim != dim0) return fail(NAUTICLE_ERR_DOMAIN, "case %d: all cases must share one dim", b);
        if (!finite_pos(q.h) || !finite_pos(q.mass) || !finite_pos(q.rho0) || !finite_pos(q.c0) ||
            !finite_pos(q.gamma) || !std::isfinite(q.nu) || q.nu < 0.0 || !std::isfinite(q.dt) || q.dt < 0.0 ||
            !std::isfinite(q.g[0]) || !std::isfinite(q.g[1]) || !std::isfinite(q.g[2]) ||
            !std::isfinite(q.alpha_av) || q.alpha_av < 0.0 || !std::isfinite(q.skin) || q.skin < 0.0)
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: non-finite or non-positive parameter", b);
        if (q.model == NAUTICLE_MODEL_SOCIAL && q.skin != 0.0)
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: the social force needs skin = 0", b);
        if (q.model < NAUTICLE_MODEL_SUMMATION || q.model > NAUTICLE_MODEL_CAHN_HILLIARD)
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: unknown model %d", b, q.model);
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(q.law[k])) return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: law[%d] not finite", b, k);
        if (q.model == NAUTICLE_MODEL_DEM && q.law[0] < 0.0)
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: friction coefficient < 0", b);
        if (q.model == NAUTICLE_MODEL_SOCIAL && (!(q.law[1] > 0.0) || !(q.law[3] > 0.0)))
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: social force needs B > 0 and tau > 0", b);
        if (q.model == NAUTICLE_MODEL_CAHN_HILLIARD && (q.law[0] < 0.0 || q.law[1] < 0.0 || !(q.law[2] > 0.0)))
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: Cahn-Hilliard needs D >= 0, gamma >= 0, factor > 0", b);
        if (q.model != model0) return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: all cases must share one model", b);
        // the lists' reach: the support plus the skin
        const double reach = 2.0 * q.h + q.skin;
        uint64_t ncell = 1;
        for (int k = 0; k < 3; ++k) {
            if (k >= d.dim) {
                if (d.ncell[k] != 1) return fail(NAUTICLE_ERR_DOMAIN, "case %d: ncell[%d] must be 1", b, k);
                continue;
            }
            if (d.ncell[k] < 1) return fail(NAUTICLE_ERR_DOMAIN, "case %d: ncell[%d] < 1", b, k);
            if (d.boundary[k] != NAUTICLE_PERIODIC && d.boundary[k] != NAUTICLE_CUTOFF &&
                d.boundary[k] != NAUTICLE_SYMMETRIC)
                return fail(NAUTICLE_ERR_DOMAIN, "case %d: boundary[%d] unknown", b, k);
            if (!finite_pos(d.cell_size[k]) || !std::isfinite(d.origin[k]))
                return fail(NAUTICLE_ERR_DOMAIN, "case %d: bad cell_size/origin on axis %d", b, k);
            const double cs32 = static_cast<double>(static_cast<float>(d.cell_size[k]));
            if (cs32 < reach)
                return fail(NAUTICLE_ERR_DOMAIN, "case %d: cell_size[%d] = %.9g below 2h + skin = %.9g", b, k,
                            cs32, reach);
            if (d.boundary[k] == NAUTICLE_PERIODIC && d.ncell[k] < 3)
                return fail(NAUTICLE_ERR_DOMAIN, "case %d: periodic axis %d needs >= 3 cells", b, k);
            // a boundary cell's images must lie beyond one face only
            if (d.boundary[k] == NAUTICLE_SYMMETRIC && d.ncell[k] < 2)
                return fail(NAUTICLE_ERR_DOMAIN, "case %d: symmetric axis %d needs >= 2 cells", b, k);
            ncell *= static_cast<uint64_t>(d.ncell[k]);
        }
        if (c.n < 0 || c.n_fixed < 0 || c.n_fixed > c.n)
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: bad n / n_fixed", b);
        if (static_cast<uint64_t>(c.offset) != n_total)
            return fail(NAUTICLE_ERR_INVALID_ARG, "case %d: offset %lld, expected %llu (contiguous)", b,
                        static_cast<long long>(c.offset), static_cast<unsigned long long>(n_total));
        CaseDev C;
        std::memset(&C, 0, sizeof(C));
        C.dim = d.dim;
        for (int k = 0; k < 3; ++k) {
            C.nc[k] = d.ncell[k];
            C.periodic[k] = (k < d.dim && d.boundary[k] == NAUTICLE_PERIODIC) ? 1 : 0;
            C.mirror[k] = (k < d.dim && d.boundary[k] == NAUTICLE_SYMMETRIC) ? 1 : 0;
            any_mirror = any_mirror || C.mirror[k];
            C.cs[k] = static_cast<float>(k < d.dim ? d.cell_size[k] : 1.0);
            C.inv_cs[k] = static_cast<float>(1.0 / (k < d.dim ? d.cell_size[k] : 1.0));
            C.origin[k] = static_cast<float>(k < d.dim ? d.origin[k] : 0.0);
            C.g[k] = static_cast<float>(k < d.dim ? q.g[k] : 0.0);
        }
        C.cell_base = static_cast<uint32_t>(n_cells_total);
        C.n_cells = static_cast<uint32_t>(ncell);
        C.offset = static_cast<uint32_t>(n_total);
        C.n = static_cast<uint32_t>(c.n);
        C.n_fluid = static_cast<uint32_t>(c.n - c.n_fixed);
        // the kernel's dimension: the domain's, or 2 for Example 1b's surface
        const int kdim = q.model == NAUTICLE_MODEL_CAHN_HILLIARD ? 2 : d.dim;
        const double alpha = kdim == 2 ? 7.0 / (4.0 * M_PI * q.h * q.h)
                                       : 21.0 / (16.0 * M_PI * q.h * q.h * q.h);
        C.R2 = static_cast<float>(reach * reach);
        {
            // a build is due once a particle has moved lim from its build-time
            // position; the margin covers the FP32 rounding of the predicate
            // and of the displacement
            double cs_max = 0.0;
            for (int k = 0; k < d.dim; ++k) cs_max = std::max(cs_max, static_cast<double>(C.cs[k]));
            const double lim = std::max(0.5 * q.skin - std::ldexp(cs_max, -18), 0.0);
            C.verlet_lim2 = static_cast<float>(lim * lim);
        }
        C.inv_h = static_cast<float>(1.0 / q.h);
        C.m = static_cast<float>(q.mass);
        C.m_alpha = static_cast<float>(q.mass * alpha);
        C.F_coef = static_cast<float>(-5.0 * alpha / (q.h * q.h));
        C.dF_coef = static_cast<float>(7.5 * alpha / (q.h * q.h * q.h));
        C.rho0 = static_cast<float>(q.rho0);
        C.inv_rho0 = static_cast<float>(1.0 / q.rho0);
        C.B = static_cast<float>(q.c0 * q.c0 * q.rho0 / q.gamma);
        C.gamma = static_cast<float>(q.gamma);
        C.c0 = static_cast<float>(q.c0);
        C.nu = static_cast<float>(q.nu);
        C.dt = static_cast<float>(q.dt);
        C.c2 = static_cast<float>(q.c0 * q.c0);
        C.h = static_cast<float>(q.h);
        for (int k = 0; k < 4; ++k) C.law[k] = static_cast<float>(q.law[k]);
        if (q.model == NAUTICLE_MODEL_CAHN_HILLIARD)  // the gradient limit of dt, gamma / (2h)^2
            C.law[3] = static_cast<float>(q.law[1] / (4.0 * q.h * q.h));
        C.av_coef = static_cast<float>(q.alpha_av * q.c0 * q.h * q.mass);
        C.item_first = static_cast<uint32_t>(D->items.size());
        for (int64_t first = 0; first < c.n; first += block) {
            Item it;
            it.case_id = static_cast<uint32_t>(b);
            it.first = static_cast<uint32_t>(n_total + first);
            it.count = static_cast<uint32_t>(std::min<int64_t>(block, c.n - first));
            it.pad = 0;
            D->items.push_back(it);
        }
        worst_items += (c.n + 63) / 64;
        // expected neighbours per particle at the case's mean number density
        double volume = 1.0;
        for (int k = 0; k < d.dim; ++k) volume *= d.ncell[k] * d.cell_size[k];
        const double ball = d.dim == 2 ? M_PI * reach * reach : 4.0 / 3.0 * M_PI * reach * reach * reach;
        nbr_per_particle.push_back(static_cast<double>(c.n) / volume * ball);
        // LDS records for an item's neighbourhood at the reference density
        // (particle volume m / rho0): 3^(dim-1) rows of the item's cells plus
        // one on each side, with 10% slack; the rest takes the global path
        double cell_volume = 1.0;
        for (int k = 0; k < d.dim; ++k) cell_volume *= d.cell_size[k];
        const double ppc = cell_volume / (q.mass / q.rho0);
        const double rows = d.dim == 3 ? 9.0 : 3.0;
        const double need = rows * (std::ceil(static_cast<double>(block) / ppc) + 3.0) * ppc * 1.1 + 32.0;
        halo_need = std::max(halo_need, need);
        C.item_count = static_cast<uint32_t>(D->items.size()) - C.item_first;
        D->cases.push_back(C);
        n_total += static_cast<uint64_t>(c.n);
        n_cells_total += ncell;
        n_fluid_total += static_cast<uint64_t>(c.n - c.n_fixed);
        if (n_total > kIndexMask)
            return fail(NAUTICLE_ERR_INVALID_ARG, "more than 2^%d particles in total", NAUTICLE_NBR_INDEX_BITS);
        if (n_cells_total >= (1ull << 31)) return fail(NAUTICLE_ERR_DOMAIN, "more than 2^31 cells in total");
    }
    P.dim_max = dim0;
    P.model = model0;
    // D->cases keeps its buffer when the plan is moved into the table of plans
    P.host_cases = D->cases.data();
    P.mirror = any_mirror ? 1u : 0u;
    P.n_total = static_cast<uint32_t>(n_total);
    P.n_cells_total = static_cast<uint32_t>(n_cells_total);
    P.n_fluid_total = static_cast<uint32_t>(n_fluid_total);
    P.n_items = static_cast<uint32_t>(D->items.size());
    P.block = static_cast<uint32_t>(block);
    P.halo_cap = static_cast<uint32_t>(std::min<double>(std::max<double>(halo_need, 256.0), 1u << 20));
    P.persistent = static_cast<uint32_t>(tn.persistent);
    int cus = 256;
    if (tn.persistent) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            return fail(NAUTICLE_ERR_HIP, "could not query the number of compute units");
    }
    P.cus = static_cast<uint32_t>(cus);
    P.groups_per_cu = static_cast<uint32_t>(tn.groups_per_cu);
    // queues: the item list cut into kXcds contiguous slices (the items a
    // grid launch gives each XCD), each slice by decreasing estimated cost
    // (particles x expected neighbours), ties in item order
    D->queue.resize(D->items.size());
    for (size_t k = 0; k < D->queue.size(); ++k) D->queue[k] = static_cast<uint32_t>(k);
    const size_t per_xcd = (D->queue.size() + kXcds - 1) / kXcds;
    for (size_t first = 0; first < D->queue.size(); first += per_xcd) {
        const size_t last = std::min(D->queue.size(), first + per_xcd);
        std::stable_sort(D->queue.begin() + first, D->queue.begin() + last, [&](uint32_t a, uint32_t b) {
            const Item& A = D->items[a];
            const Item& B = D->items[b];
            return A.count * nbr_per_particle[A.case_id] > B.count * nbr_per_particle[B.case_id];
        });
    }
    int bits = 1;
    while ((1ull << bits) < n_cells_total) ++bits;
    P.key_bits = bits;
    P.fingerprint = fingerprint(cases, n_cases);

    // workspace layout
    Layout& L = P.L;
    const size_t N = std::max<size_t>(n_total, 1);
    const size_t n_tiles = (N + kSortTile - 1) / kSortTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.err = take(sizeof(uint32_t));
    L.cases = take(sizeof(CaseDev) * D->cases.size());
    const size_t n_items_max = std::max<size_t>(static_cast<size_t>(worst_items), 1);
    L.items = take(sizeof(Item) * n_items_max);
    L.queue = take(sizeof(uint32_t) * n_items_max);
    L.counters = take(sizeof(uint32_t) * kCounters * kXcds * kCounterStride);
    for (int k = 0; k < 9; ++k) L.state[k] = take(4 * N);
    L.sort_keys = take(4 * N);
    L.sort_vals = take(4 * N);
    L.sort_hist = take(4 * kSortBins * n_tiles);
    L.sort_totals = take(4 * kSortBins);
    L.cell_first = take(4 * (static_cast<size_t>(n_cells_total) + 1));
    L.pos4 = take(16 * (N + kPosPad));
    L.a4 = take(16 * N);
    L.b4 = take(16 * N);
    L.adj4 = take(16 * N);
    L.adj2 = take(8 * N);
    L.adj4b = take(16 * N);
    L.vr4 = model0 == NAUTICLE_MODEL_CONTINUITY ? take(16 * N) : 0;
    L.chmax = take(sizeof(float) * n_items_max);
    L.partial = take(2 * sizeof(double) * n_items_max);
    L.inv_map = take(4 * N);
    const bool moving = model0 == NAUTICLE_MODEL_SUMMATION || model0 == NAUTICLE_MODEL_CONTINUITY ||
                        model0 == NAUTICLE_MODEL_DEM;
    for (int k = 0; k < 3; ++k) L.off0[k] = moving && k < dim0 ? take(4 * N) : 0;
    L.vflag = take(2 * sizeof(uint32_t));
    L.total = off;
    return NAUTICLE_OK;
}

std::mutex g_mu;
std::unordered_map<const void*, Derived> g_plans;

// Looks up the plan recorded for ws and checks it matches the given cases.
nauticle_status plan_for(const nauticle_case* cases, int32_t n_cases, void* ws, size_t ws_bytes,
                         const Plan** out)
{
    if (!cases || n_cases < 1) return fail(NAUTICLE_ERR_INVALID_ARG, "cases is null or n_cases < 1");
    if (!ws) return fail(NAUTICLE_ERR_WORKSPACE, "workspace is null");
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_plans.find(ws);
    if (it == g_plans.end()) return fail(NAUTICLE_ERR_WORKSPACE, "workspace was not prepared (nauticle_prepare)");
    const Plan& P = it->second.plan;
    if (P.n_cases != n_cases || P.fingerprint != fingerprint(cases, n_cases))
        return fail(NAUTICLE_ERR_WORKSPACE, "workspace was prepared for a different case table");
    if (ws_bytes < P.L.total) return fail(NAUTICLE_ERR_WORKSPACE, "workspace too small");
    *out = &P;
    return NAUTICLE_OK;
}

nauticle_status check_state(const Plan& P, const nauticle_state* st, bool need_vel, const char* name,
                            bool need_rho = false)
{
    if (!st) return fail(NAUTICLE_ERR_INVALID_ARG, "%s is null", name);
    if (P.n_total == 0) return NAUTICLE_OK;
    if (!st->cell || !st->id) return fail(NAUTICLE_ERR_INVALID_ARG, "%s: cell/id null", name);
    if (need_rho && !st->rho) return fail(NAUTICLE_ERR_INVALID_ARG, "%s: rho null (continuity model)", name);
    for (int k = 0; k < P.dim_max; ++k) {
        if (!st->off[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "%s: off[%d] null", name, k);
        if (need_vel && !st->vel[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "%s: vel[%d] null", name, k);
    }
    return NAUTICLE_OK;
}

nauticle_status check_cells(const Plan& P, const nauticle_cells* c, bool need_lists)
{
    if (!c) return fail(NAUTICLE_ERR_INVALID_ARG, "cells is null");
    if (c->max_nbr < kChunk || c->max_nbr > 1024 || c->max_nbr % kChunk != 0)
        return fail(NAUTICLE_ERR_INVALID_ARG, "max_nbr must be a multiple of 4 in [4, 1024]");
    if (!c->cell_start || !c->cell_end) return fail(NAUTICLE_ERR_INVALID_ARG, "cell_start/end null");
    if (P.n_total == 0) return NAUTICLE_OK;
    if (!c->key || !c->perm) return fail(NAUTICLE_ERR_INVALID_ARG, "key/perm null");
    if (need_lists && (!c->nbr || !c->nbr_count)) return fail(NAUTICLE_ERR_INVALID_ARG, "nbr/nbr_count null");
    if (need_lists && reinterpret_cast<uintptr_t>(c->nbr) % 16 != 0)
        return fail(NAUTICLE_ERR_INVALID_ARG, "nbr must be 16-byte aligned");
    if (static_cast<uint64_t>(c->max_nbr) * P.n_total > (1ull << 40))
        return fail(NAUTICLE_ERR_INVALID_ARG, "neighbour list too large");
    return NAUTICLE_OK;
}

nauticle_status check_fields(const Plan& P, const nauticle_fields* f, bool need_acc)
{
    if (!f) return fail(NAUTICLE_ERR_INVALID_ARG, "fields is null");
    if (P.n_total == 0) return NAUTICLE_OK;
    if (!f->rho || !f->p || !f->s || !f->inv_rho) return fail(NAUTICLE_ERR_INVALID_ARG, "fields: null array");
    if (need_acc)
        for (int k = 0; k < P.dim_max; ++k)
            if (!f->acc[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "fields: acc[%d] null", k);
    return NAUTICLE_OK;
}

StateDev to_dev(const nauticle_state* s)
{
    StateDev d;
    d.cell = s->cell;
    d.id = s->id;
    for (int k = 0; k < 3; ++k) {
        d.off[k] = s->off[k];
        d.vel[k] = s->vel[k];
    }
    d.rho = s->rho;
    return d;
}

// The state as the plan's model reads it: rho only for the continuity model.
StateDev to_dev_model(const Plan& P, const nauticle_state* s)
{
    StateDev d = to_dev(s);
    if (P.model != NAUTICLE_MODEL_CONTINUITY) d.rho = nullptr;
    return d;
}

FieldsDev to_dev(const nauticle_fields* f)
{
    FieldsDev d;
    d.rho = f->rho;
    d.p = f->p;
    d.s = f->s;
    d.inv_rho = f->inv_rho;
    for (int k = 0; k < 3; ++k) d.acc[k] = f->acc[k];
    d.drho = f->drho;
    return d;
}

StateDev scratch_state(const Plan& P, void* ws)
{
    StateDev d;
    d.cell = at<uint32_t>(ws, P.L.state[0]);
    for (int k = 0; k < 3; ++k) {
        d.off[k] = at<float>(ws, P.L.state[1 + k]);
        d.vel[k] = at<float>(ws, P.L.state[4 + k]);
    }
    d.id = at<uint32_t>(ws, P.L.state[7]);
    d.rho = P.model == NAUTICLE_MODEL_CONTINUITY ? at<float>(ws, P.L.state[8]) : nullptr;
    return d;
}

}  // namespace

extern "C" {

int64_t nauticle_cells_total(const nauticle_case* cases, int32_t n_cases)
{
    if (!cases || n_cases < 1) return -1;
    int64_t total = 0;
    for (int32_t b = 0; b < n_cases; ++b) {
        int64_t c = 1;
        for (int k = 0; k < 3; ++k) c *= std::max<int64_t>(cases[b].dom.ncell[k], 0);
        total += c;
    }
    return total;
}

nauticle_status nauticle_workspace_bytes(const nauticle_case* cases, int32_t n_cases, size_t* bytes)
{
    if (!bytes) return fail(NAUTICLE_ERR_INVALID_ARG, "bytes is null");
    Derived D;
    nauticle_status st = derive(cases, n_cases, nullptr, &D);
    if (st != NAUTICLE_OK) return st;
    *bytes = D.plan.L.total;
    return NAUTICLE_OK;
}

nauticle_status nauticle_prepare(const nauticle_case* cases, int32_t n_cases, const nauticle_tuning* tuning,
                                 void* ws, size_t ws_bytes, hipStream_t stream)
{
    Derived D;
    nauticle_status st = derive(cases, n_cases, tuning, &D);
    if (st != NAUTICLE_OK) return st;
    if (!ws) return fail(NAUTICLE_ERR_WORKSPACE, "workspace is null");
    if (ws_bytes < D.plan.L.total)
        return fail(NAUTICLE_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, D.plan.L.total);
    hipError_t e = hipMemsetAsync(at<char>(ws, D.plan.L.err), 0, sizeof(uint32_t), stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<char>(ws, D.plan.L.cases), D.cases.data(), sizeof(CaseDev) * D.cases.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !D.items.empty())
        e = hipMemcpyAsync(at<char>(ws, D.plan.L.items), D.items.data(), sizeof(Item) * D.items.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !D.queue.empty())
        e = hipMemcpyAsync(at<char>(ws, D.plan.L.queue), D.queue.data(), sizeof(uint32_t) * D.queue.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "nauticle_prepare upload");
    std::lock_guard<std::mutex> lock(g_mu);
    g_plans[ws] = std::move(D);
    return NAUTICLE_OK;
}

nauticle_status nauticle_bin(const nauticle_case* cases, int32_t n_cases, const float* const pos[3],
                             nauticle_state* state, void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, state, false, "state")) != NAUTICLE_OK) return st;
    if (!pos) return fail(NAUTICLE_ERR_INVALID_ARG, "pos is null");
    for (int k = 0; k < P->dim_max; ++k)
        if (P->n_total && !pos[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "pos[%d] is null", k);
    hipError_t e = launch_bin(*P, ws, pos, to_dev(state), stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_bin");
}

nauticle_status nauticle_unbin(const nauticle_case* cases, int32_t n_cases, const nauticle_state* state,
                               float* const pos[3], void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, state, false, "state")) != NAUTICLE_OK) return st;
    if (!pos) return fail(NAUTICLE_ERR_INVALID_ARG, "pos is null");
    for (int k = 0; k < P->dim_max; ++k)
        if (P->n_total && !pos[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "pos[%d] is null", k);
    hipError_t e = launch_unbin(*P, ws, to_dev(state), pos, false, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_unbin");
}

nauticle_status nauticle_unbin_by_id(const nauticle_case* cases, int32_t n_cases, const nauticle_state* state,
                                     float* const pos[3], void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, state, false, "state")) != NAUTICLE_OK) return st;
    if (!pos) return fail(NAUTICLE_ERR_INVALID_ARG, "pos is null");
    for (int k = 0; k < P->dim_max; ++k)
        if (P->n_total && !pos[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "pos[%d] is null", k);
    hipError_t e = launch_unbin(*P, ws, to_dev(state), pos, true, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_unbin_by_id");
}

nauticle_status nauticle_gather_by_id(const nauticle_case* cases, int32_t n_cases, const nauticle_state* state,
                                      const float* const g[3], float* const out[3], void* ws, size_t ws_bytes,
                                      hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if (!state || (P->n_total && !state->id)) return fail(NAUTICLE_ERR_INVALID_ARG, "state or state->id is null");
    if (!g || !out) return fail(NAUTICLE_ERR_INVALID_ARG, "g or out is null");
    for (int k = 0; k < P->dim_max; ++k) {
        if (P->n_total && (!g[k] || !out[k])) return fail(NAUTICLE_ERR_INVALID_ARG, "g[%d] or out[%d] is null", k, k);
        for (int j = 0; j < P->dim_max; ++j)
            if (P->n_total && out[k] == g[j]) return fail(NAUTICLE_ERR_INVALID_ARG, "out must not alias g");
    }
    hipError_t e = launch_gather_id(*P, ws, state->id, g, out, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_gather_by_id");
}

nauticle_status nauticle_build_cells(const nauticle_case* cases, int32_t n_cases, const nauticle_state* in,
                                     nauticle_state* sorted, nauticle_cells* cells, void* ws, size_t ws_bytes,
                                     hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    const bool cont = P->model == NAUTICLE_MODEL_CONTINUITY;
    if ((st = check_state(*P, in, true, "in", cont)) != NAUTICLE_OK) return st;
    if ((st = check_state(*P, sorted, true, "sorted", cont)) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if (P->n_total && (in->cell == sorted->cell || in->off[0] == sorted->off[0] || (cont && in->rho == sorted->rho)))
        return fail(NAUTICLE_ERR_INVALID_ARG, "sorted must not alias in");
    hipError_t e = launch_build_cells(*P, ws, to_dev_model(*P, in), to_dev_model(*P, sorted), *cells, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_build_cells");
}

nauticle_status nauticle_sph_density(const nauticle_case* cases, int32_t n_cases, const nauticle_state* sorted,
                                     const nauticle_cells* cells, nauticle_fields* fields, void* ws,
                                     size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, sorted, false, "sorted")) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_fields(*P, fields, false)) != NAUTICLE_OK) return st;
    hipError_t e = launch_cell_first(*P, ws, *cells, stream);
    if (e == hipSuccess) e = launch_pack_positions(*P, ws, to_dev(sorted), stream);
    if (e == hipSuccess) e = launch_density(*P, ws, to_dev(sorted), *cells, to_dev(fields), stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_sph_density");
}

nauticle_status nauticle_sph_continuity(const nauticle_case* cases, int32_t n_cases, const nauticle_state* sorted,
                                        const nauticle_cells* cells, nauticle_fields* fields, void* ws,
                                        size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if (P->model != NAUTICLE_MODEL_CONTINUITY)
        return fail(NAUTICLE_ERR_INVALID_ARG, "nauticle_sph_continuity needs the continuity model");
    if ((st = check_state(*P, sorted, true, "sorted", true)) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_fields(*P, fields, false)) != NAUTICLE_OK) return st;
    if (P->n_total && fields->rho == sorted->rho)
        return fail(NAUTICLE_ERR_INVALID_ARG, "fields->rho must not alias sorted->rho");
    const StateDev sd = to_dev(sorted);
    hipError_t e = launch_cell_first(*P, ws, *cells, stream);
    if (e == hipSuccess) e = launch_pack_positions(*P, ws, sd, stream);
    if (e == hipSuccess) e = launch_pack_continuity(*P, ws, sd, stream);
    if (e == hipSuccess) e = launch_continuity(*P, ws, sd, *cells, to_dev(fields), stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_sph_continuity");
}

namespace {

bool is_law(const Plan& P) { return P.model == NAUTICLE_MODEL_DEM || P.model == NAUTICLE_MODEL_SOCIAL; }

nauticle_status check_attrs(const Plan& P, const nauticle_law_attrs* a, LawAttrsDev* out)
{
    if (!a) return fail(NAUTICLE_ERR_INVALID_ARG, "attrs is null");
    if (P.n_total && (!a->radius || !a->mass || !a->coef))
        return fail(NAUTICLE_ERR_INVALID_ARG, "attrs: radius/mass/coef null");
    if (P.n_total && P.model == NAUTICLE_MODEL_SOCIAL) {
        if (!a->v0) return fail(NAUTICLE_ERR_INVALID_ARG, "attrs: v0 null (social force)");
        for (int k = 0; k < P.dim_max; ++k)
            if (!a->goal[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "attrs: goal[%d] null (social force)", k);
    }
    out->radius = a->radius;
    out->mass = a->mass;
    out->coef = a->coef;
    out->v0 = a->v0;
    for (int k = 0; k < 3; ++k) out->goal[k] = a->goal[k];
    return NAUTICLE_OK;
}

nauticle_status check_acc(const Plan& P, const nauticle_fields* f)
{
    if (!f) return fail(NAUTICLE_ERR_INVALID_ARG, "fields is null");
    for (int k = 0; k < P.dim_max; ++k)
        if (P.n_total && !f->acc[k]) return fail(NAUTICLE_ERR_INVALID_ARG, "fields: acc[%d] null", k);
    return NAUTICLE_OK;
}

}  // namespace

nauticle_status nauticle_interact(const nauticle_case* cases, int32_t n_cases, const nauticle_state* sorted,
                                  const nauticle_cells* cells, const nauticle_law_attrs* attrs, nauticle_fields* fields,
                                  nauticle_state* next, void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if (!is_law(*P)) return fail(NAUTICLE_ERR_INVALID_ARG, "nauticle_interact needs a DEM or social-force table");
    LawAttrsDev ad;
    if ((st = check_state(*P, sorted, true, "sorted")) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_attrs(*P, attrs, &ad)) != NAUTICLE_OK) return st;
    if ((st = check_acc(*P, fields)) != NAUTICLE_OK) return st;
    StateDev nd;
    if (next) {
        if ((st = check_state(*P, next, true, "next")) != NAUTICLE_OK) return st;
        if (P->n_total && (next->cell == sorted->cell || next->off[0] == sorted->off[0]))
            return fail(NAUTICLE_ERR_INVALID_ARG, "next must not alias sorted");
        nd = to_dev_model(*P, next);
    }
    hipError_t e = launch_cell_first(*P, ws, *cells, stream);
    if (e == hipSuccess)
        e = launch_interact(*P, ws, to_dev_model(*P, sorted), *cells, ad, to_dev(fields), next ? &nd : nullptr, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_interact");
}

nauticle_status nauticle_step_law(const nauticle_case* cases, int32_t n_cases, nauticle_state* state, int32_t n_steps,
                                  nauticle_cells* cells, nauticle_fields* fields, const nauticle_law_attrs* attrs,
                                  hipEvent_t* phase_events, void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if (!is_law(*P)) return fail(NAUTICLE_ERR_INVALID_ARG, "nauticle_step_law needs a DEM or social-force table");
    if (n_steps < 0) return fail(NAUTICLE_ERR_INVALID_ARG, "n_steps < 0");
    LawAttrsDev ad;
    if ((st = check_state(*P, state, true, "state")) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_attrs(*P, attrs, &ad)) != NAUTICLE_OK) return st;
    if ((st = check_acc(*P, fields)) != NAUTICLE_OK) return st;
    const StateDev cur = to_dev_model(*P, state);
    const StateDev tmp = scratch_state(*P, ws);
    const FieldsDev f = to_dev(fields);
    auto mark = [&](int32_t s, int k) {
        return phase_events ? hipEventRecord(phase_events[5 * s + k], stream) : hipSuccess;
    };
    for (int32_t s = 0; s < n_steps; ++s) {
        hipError_t e = mark(s, 0);
        if (e == hipSuccess)
            e = launch_build_cells(*P, ws, cur, tmp, *cells, stream, phase_events ? phase_events[5 * s + 1] : nullptr);
        if (e == hipSuccess) e = mark(s, 2);
        if (e == hipSuccess) e = mark(s, 3);
        if (e == hipSuccess) e = launch_interact(*P, ws, tmp, *cells, ad, f, &cur, stream);
        if (e == hipSuccess) e = mark(s, 4);
        if (e != hipSuccess) return hip_fail(e, "nauticle_step_law");
    }
    return NAUTICLE_OK;
}

nauticle_status nauticle_ch_steps(const nauticle_case* cases, int32_t n_cases, const nauticle_state* sorted,
                                  const nauticle_cells* cells, float* c, float* mu, float* cdot, double* clock,
                                  int32_t n_steps, void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if (P->model != NAUTICLE_MODEL_CAHN_HILLIARD)
        return fail(NAUTICLE_ERR_INVALID_ARG, "nauticle_ch_steps needs a Cahn-Hilliard table");
    if (n_steps < 0) return fail(NAUTICLE_ERR_INVALID_ARG, "n_steps < 0");
    if ((st = check_state(*P, sorted, false, "sorted")) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if (!clock) return fail(NAUTICLE_ERR_INVALID_ARG, "clock is null");
    if (P->n_total && !c) return fail(NAUTICLE_ERR_INVALID_ARG, "c is null");
    if (P->n_total && (c == mu || c == cdot || (mu && mu == cdot)))
        return fail(NAUTICLE_ERR_INVALID_ARG, "c, mu and cdot must be distinct");
    hipError_t e = launch_ch_steps(*P, ws, to_dev_model(*P, sorted), *cells, c, mu, cdot, clock, n_steps, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_ch_steps");
}

nauticle_status nauticle_sph_forces(const nauticle_case* cases, int32_t n_cases, const nauticle_state* sorted,
                                    const nauticle_cells* cells, nauticle_fields* fields, nauticle_state* next,
                                    void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, sorted, true, "sorted")) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_fields(*P, fields, true)) != NAUTICLE_OK) return st;
    StateDev nd;
    if (next) {
        const bool cont = P->model == NAUTICLE_MODEL_CONTINUITY;
        if ((st = check_state(*P, next, true, "next", cont)) != NAUTICLE_OK) return st;
        if (P->n_total && (next->cell == sorted->cell || next->off[0] == sorted->off[0]))
            return fail(NAUTICLE_ERR_INVALID_ARG, "next must not alias sorted");
        nd = to_dev_model(*P, next);
    }
    hipError_t e = launch_cell_first(*P, ws, *cells, stream);
    if (e == hipSuccess) e = launch_pack_fields(*P, ws, to_dev_model(*P, sorted), to_dev(fields), stream);
    if (e == hipSuccess)
        e = launch_forces(*P, ws, to_dev_model(*P, sorted), *cells, to_dev(fields), next ? &nd : nullptr, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_sph_forces");
}

}  // extern "C"

namespace {

// Host-side checks of nauticle_step's arguments against a plan.
nauticle_status check_step_args(const Plan* P, const nauticle_state* state, int32_t n_steps,
                                const nauticle_cells* cells, const nauticle_fields* fields)
{
    nauticle_status st;
    if (n_steps < 0) return fail(NAUTICLE_ERR_INVALID_ARG, "n_steps < 0");
    if (is_law(*P)) return fail(NAUTICLE_ERR_INVALID_ARG, "pair-law tables step with nauticle_step_law");
    if (P->model == NAUTICLE_MODEL_CAHN_HILLIARD)
        return fail(NAUTICLE_ERR_INVALID_ARG, "Cahn-Hilliard tables step with nauticle_ch_steps");
    const bool cont = P->model == NAUTICLE_MODEL_CONTINUITY;
    if ((st = check_state(*P, state, true, "state", cont)) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_fields(*P, fields, true)) != NAUTICLE_OK) return st;
    return NAUTICLE_OK;
}

// The launch sequence of nauticle_step on a checked plan and workspace.
nauticle_status run_steps(const Plan* P, nauticle_state* state, int32_t n_steps, nauticle_cells* cells,
                          nauticle_fields* fields, hipEvent_t* phase_events, void* ws, hipStream_t stream,
                          nauticle_state* sorted_out = nullptr)
{
    const bool cont = P->model == NAUTICLE_MODEL_CONTINUITY;
    const StateDev cur = to_dev_model(*P, state);
    // the sorted copy: the caller's, or the workspace's
    const StateDev tmp = sorted_out ? to_dev_model(*P, sorted_out) : scratch_state(*P, ws);
    const FieldsDev f = to_dev(fields);
    // build_cells leaves packed positions for density, and density leaves
    // packed fields for forces, so the step needs no separate packing
    auto mark = [&](int32_t s, int k) {
        return phase_events ? hipEventRecord(phase_events[5 * s + k], stream) : hipSuccess;
    };
    for (int32_t s = 0; s < n_steps; ++s) {
        hipError_t e = mark(s, 0);
        if (e == hipSuccess)
            e = launch_build_cells(*P, ws, cur, tmp, *cells, stream, phase_events ? phase_events[5 * s + 1] : nullptr);
        if (e == hipSuccess) e = mark(s, 2);
        if (cont) {
            if (e == hipSuccess) e = launch_pack_continuity(*P, ws, tmp, stream);
            if (e == hipSuccess) e = launch_continuity(*P, ws, tmp, *cells, f, stream);
        } else if (e == hipSuccess) {
            e = launch_density(*P, ws, tmp, *cells, f, stream);
        }
        if (e == hipSuccess) e = mark(s, 3);
        if (e == hipSuccess) e = launch_forces(*P, ws, tmp, *cells, f, &cur, stream);
        if (e == hipSuccess) e = mark(s, 4);
        if (e != hipSuccess) return hip_fail(e, "nauticle_step");
    }
    return NAUTICLE_OK;
}

}  // namespace

// Fixed device scratch of nauticle_step_fixed_scratch: a workspace that
// lives in the code object, so that the entry point needs no allocation.
// One copy per device (each at its own address), held until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy:
// its name on the host is a stand-in, not the device address; the address
// comes from hipGetSymbolAddress, once per device.
static constexpr size_t kFixedScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (looked up on its first use).
nauticle_status fixed_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(NAUTICLE_ERR_INVALID_ARG, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(NAUTICLE_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return NAUTICLE_OK;
}

// Reads and clears the error word of a workspace after the stream has drained.
nauticle_status drain_and_read_error(const Plan& P, void* ws, hipStream_t stream, const char* where)
{
    uint32_t word = 0;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&word, at<char>(ws, P.L.err), sizeof(word), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, where);
    if (word & kErrNonFinite) return fail(NAUTICLE_ERR_NONFINITE, "a non-finite value was produced or given");
    if (word & kErrOverflow) return fail(NAUTICLE_ERR_NEIGHBOUR_OVERFLOW, "a particle had more than max_nbr neighbours");
    if (word & kErrOutOfDomain) return fail(NAUTICLE_ERR_OUT_OF_DOMAIN, "a position lies beyond 2^23 cells");
    if (word & kErrAttribute) return fail(NAUTICLE_ERR_ATTRIBUTE, "a pair-law attribute is out of range");
    return NAUTICLE_OK;
}

}  // namespace

extern "C" {

nauticle_status nauticle_step(const nauticle_case* cases, int32_t n_cases, nauticle_state* state, int32_t n_steps,
                              nauticle_cells* cells, nauticle_fields* fields, hipEvent_t* phase_events, void* ws,
                              size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_step_args(P, state, n_steps, cells, fields)) != NAUTICLE_OK) return st;
    return run_steps(P, state, n_steps, cells, fields, phase_events, ws, stream);
}

nauticle_status nauticle_step_record(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                     nauticle_state* sorted, nauticle_cells* cells, nauticle_fields* fields,
                                     void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_step_args(P, state, 1, cells, fields)) != NAUTICLE_OK) return st;
    const bool cont = P->model == NAUTICLE_MODEL_CONTINUITY;
    if ((st = check_state(*P, sorted, true, "sorted", cont)) != NAUTICLE_OK) return st;
    if (P->n_total > 0 && (sorted->cell == state->cell || sorted->id == state->id))
        return fail(NAUTICLE_ERR_INVALID_ARG, "sorted must not share arrays with state");
    return run_steps(P, state, 1, cells, fields, nullptr, ws, stream, sorted);
}

nauticle_status nauticle_step_cfl(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                  int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields, double cfl,
                                  double* clock, void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_step_args(P, state, n_steps, cells, fields)) != NAUTICLE_OK) return st;
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(NAUTICLE_ERR_INVALID_ARG, "cfl must be finite and > 0");
    if (!clock) return fail(NAUTICLE_ERR_INVALID_ARG, "clock is null");
    // the host copy of the device case table: its fixed time steps are put
    // back at the end, so that later calls on the workspace use them
    const void* table = nullptr;
    size_t table_bytes = 0;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        const Derived& D = g_plans.at(ws);
        table = D.cases.data();
        table_bytes = sizeof(CaseDev) * D.cases.size();
    }
    for (int32_t s = 0; s < n_steps; ++s) {
        hipError_t e = launch_cfl(*P, ws, to_dev_model(*P, state), cfl, clock, stream);
        if (e != hipSuccess) return hip_fail(e, "nauticle_step_cfl");
        if ((st = run_steps(P, state, 1, cells, fields, nullptr, ws, stream)) != NAUTICLE_OK) return st;
    }
    hipError_t e = hipMemcpyAsync(at<char>(ws, P->L.cases), table, table_bytes, hipMemcpyHostToDevice, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_step_cfl restore");
}

nauticle_status nauticle_step_fixed_scratch(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                            int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields,
                                            hipStream_t stream)
{
    Derived D;
    nauticle_status st = derive(cases, n_cases, nullptr, &D);
    if (st != NAUTICLE_OK) return st;
    if (D.plan.L.total > kFixedScratchBytes)
        return fail(NAUTICLE_ERR_WORKSPACE, "nauticle_step_fixed_scratch: these cases need %zu bytes of scratch, "
                    "the fixed scratch holds %zu", D.plan.L.total, kFixedScratchBytes);
    if ((st = check_step_args(&D.plan, state, n_steps, cells, fields)) != NAUTICLE_OK) return st;
    void* ws = nullptr;
    if ((st = fixed_scratch(&ws)) != NAUTICLE_OK) return st;
    // the scratch keeps the last call's contents: the error word starts at
    // zero, the case table and work lists are written anew (the persistent
    // queue counters are zeroed by the launches themselves; this table runs
    // grid launches)
    hipError_t e = hipMemsetAsync(at<char>(ws, D.plan.L.err), 0, sizeof(uint32_t), stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<char>(ws, D.plan.L.cases), D.cases.data(), sizeof(CaseDev) * D.cases.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !D.items.empty())
        e = hipMemcpyAsync(at<char>(ws, D.plan.L.items), D.items.data(), sizeof(Item) * D.items.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !D.queue.empty())
        e = hipMemcpyAsync(at<char>(ws, D.plan.L.queue), D.queue.data(), sizeof(uint32_t) * D.queue.size(),
                           hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "nauticle_step_fixed_scratch upload");
    st = run_steps(&D.plan, state, n_steps, cells, fields, nullptr, ws, stream);
    // the host copies of the table must outlive the uploads: drain before returning
    const nauticle_status dev = drain_and_read_error(D.plan, ws, stream, "nauticle_step_fixed_scratch");
    return st != NAUTICLE_OK ? st : dev;
}

nauticle_status nauticle_step_verlet(const nauticle_case* cases, int32_t n_cases, nauticle_state* state,
                                     int32_t n_steps, nauticle_cells* cells, nauticle_fields* fields,
                                     const nauticle_law_attrs* attrs, int32_t* n_builds, hipEvent_t* phase_events,
                                     void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if (n_steps < 0) return fail(NAUTICLE_ERR_INVALID_ARG, "n_steps < 0");
    const bool dem = P->model == NAUTICLE_MODEL_DEM;
    if (P->model != NAUTICLE_MODEL_SUMMATION && P->model != NAUTICLE_MODEL_CONTINUITY && !dem)
        return fail(NAUTICLE_ERR_INVALID_ARG, "nauticle_step_verlet needs a SUMMATION, CONTINUITY or DEM table");
    const bool cont = P->model == NAUTICLE_MODEL_CONTINUITY;
    LawAttrsDev ad{};
    if ((st = check_state(*P, state, true, "state", cont)) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = dem ? check_acc(*P, fields) : check_fields(*P, fields, true)) != NAUTICLE_OK) return st;
    if (dem && (st = check_attrs(*P, attrs, &ad)) != NAUTICLE_OK) return st;
    if (n_builds) *n_builds = 0;
    if (n_steps == 0) return NAUTICLE_OK;
    // the rebuild word comes back through a pinned host word (one per host
    // thread, kept until the process ends), so the copy does not block
    thread_local uint32_t* t_word = nullptr;
    if (!t_word) {
        hipError_t a = hipHostMalloc(reinterpret_cast<void**>(&t_word), sizeof(uint32_t), hipHostMallocDefault);
        if (a != hipSuccess) {
            t_word = nullptr;
            return hip_fail(a, "nauticle_step_verlet: pinned host word");
        }
    }
    hipEvent_t copied;
    hipError_t e = hipEventCreateWithFlags(&copied, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "nauticle_step_verlet: event");
    const StateDev cur = to_dev_model(*P, state);
    const StateDev tmp = scratch_state(*P, ws);
    const FieldsDev f = to_dev(fields);
    const uint32_t* flag = at<uint32_t>(ws, P->L.vflag);
    auto mark = [&](int32_t s, int k) {
        return phase_events ? hipEventRecord(phase_events[5 * s + k], stream) : hipSuccess;
    };
    // the step's first pass: density or continuity (SPH), the contact pass (DEM; its records are
    // packed at a build, and between builds the drift keeps them current)
    auto first_pass = [&](bool after_build) -> hipError_t {
        if (dem)
            return after_build ? launch_interact(*P, ws, tmp, *cells, ad, f, nullptr, stream)
                               : launch_interact_on_records(*P, ws, tmp, *cells, ad, f, stream);
        if (cont) {
            hipError_t r = launch_pack_continuity(*P, ws, tmp, stream);
            return r == hipSuccess ? launch_continuity(*P, ws, tmp, *cells, f, stream) : r;
        }
        return launch_density(*P, ws, tmp, *cells, f, stream);
    };
    // Without phase events, the next step's first pass is queued before the
    // host waits for the rebuild word, so the device does not idle during the
    // round trip.  It reads the state and writes only fields and packed
    // records, so when a build turns out to be due its work is redone after
    // the build.
    const bool ahead_ok = phase_events == nullptr;
    bool ahead = false;  // this step's first pass was queued at the end of the previous one
    int32_t builds = 0;
    bool build = true;
    e = launch_verlet_clear(*P, ws, stream);
    // the live state is the workspace copy `tmp` (sorted order of the last
    // build, offsets drifting); `state` receives it re-split before each
    // build and at the end
    for (int32_t s = 0; s < n_steps && e == hipSuccess; ++s) {
        e = mark(s, 0);
        if (build) {
            if (e == hipSuccess && builds > 0) e = launch_resplit(*P, ws, tmp, cur, stream);
            if (e == hipSuccess)
                e = launch_build_cells(*P, ws, cur, tmp, *cells, stream, phase_events ? phase_events[5 * s + 1] : nullptr);
            ++builds;
        } else if (e == hipSuccess) {
            e = mark(s, 1);
        }
        if (e == hipSuccess) e = mark(s, 2);
        if (dem) {
            if (e == hipSuccess) e = mark(s, 3);
            if (e == hipSuccess && !ahead) e = first_pass(build);
        } else {
            if (e == hipSuccess && !ahead) e = first_pass(build);
            if (e == hipSuccess) e = mark(s, 3);
            if (e == hipSuccess) e = launch_forces(*P, ws, tmp, *cells, f, nullptr, stream);
        }
        if (e == hipSuccess) e = launch_verlet_drift(*P, ws, tmp, f, build, s & 1, stream);
        if (e == hipSuccess) e = mark(s, 4);
        ahead = false;
        if (e == hipSuccess && s + 1 < n_steps) {
            // is a build due before the next step?
            e = hipMemcpyAsync(t_word, flag + (s & 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipEventRecord(copied, stream);
            if (e == hipSuccess && ahead_ok) e = first_pass(false);
            if (e == hipSuccess) e = hipEventSynchronize(copied);
            build = *t_word != 0u;
            ahead = ahead_ok && !build;
        }
    }
    if (e == hipSuccess) e = launch_resplit(*P, ws, tmp, cur, stream);
    const hipError_t d = hipEventDestroy(copied);
    if (e == hipSuccess) e = d;
    if (e != hipSuccess) return hip_fail(e, "nauticle_step_verlet");
    if (n_builds) *n_builds = builds;
    return NAUTICLE_OK;
}

nauticle_status nauticle_sph_adjoint(const nauticle_case* cases, int32_t n_cases, const nauticle_state* sorted,
                                     const nauticle_cells* cells, const nauticle_fields* fields,
                                     const float* const lam_x_next[3], const float* const lam_v_next[3],
                                     float* const lam_x[3], float* const lam_v[3], double* dnu, double* dc0,
                                     void* ws, size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, sorted, true, "sorted")) != NAUTICLE_OK) return st;
    if ((st = check_cells(*P, cells, true)) != NAUTICLE_OK) return st;
    if ((st = check_fields(*P, fields, false)) != NAUTICLE_OK) return st;
    if (P->mirror || P->model != NAUTICLE_MODEL_SUMMATION)
        return fail(NAUTICLE_ERR_INVALID_ARG, "adjoint: only the summation model without symmetric faces");
    if (!lam_x_next || !lam_v_next || !lam_x || !lam_v || !dnu || !dc0)
        return fail(NAUTICLE_ERR_INVALID_ARG, "adjoint: null argument");
    for (int k = 0; k < P->dim_max; ++k) {
        if (P->n_total && (!lam_x_next[k] || !lam_v_next[k] || !lam_x[k] || !lam_v[k]))
            return fail(NAUTICLE_ERR_INVALID_ARG, "adjoint: null cotangent array on axis %d", k);
        if (P->n_total && (lam_x[k] == lam_x_next[k] || lam_v[k] == lam_v_next[k] ||
                           lam_x[k] == lam_v_next[k] || lam_v[k] == lam_x_next[k]))
            return fail(NAUTICLE_ERR_INVALID_ARG, "adjoint: outputs must not alias inputs");
    }
    hipError_t e = launch_adjoint(*P, ws, to_dev(sorted), *cells, to_dev(const_cast<nauticle_fields*>(fields)),
                                  lam_x_next, lam_v_next, lam_x, lam_v, dnu, dc0, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_sph_adjoint");
}

nauticle_status nauticle_position_loss(const nauticle_case* cases, int32_t n_cases, const nauticle_state* a,
                                       const nauticle_state* b, double* loss, float* const grad[3], void* ws,
                                       size_t ws_bytes, hipStream_t stream)
{
    const Plan* P;
    nauticle_status st = plan_for(cases, n_cases, ws, ws_bytes, &P);
    if (st != NAUTICLE_OK) return st;
    if ((st = check_state(*P, a, false, "a")) != NAUTICLE_OK) return st;
    if ((st = check_state(*P, b, false, "b")) != NAUTICLE_OK) return st;
    if (!loss) return fail(NAUTICLE_ERR_INVALID_ARG, "loss is null");
    hipError_t e = launch_position_loss(*P, ws, to_dev(a), to_dev(b), loss, grad, stream);
    return e == hipSuccess ? NAUTICLE_OK : hip_fail(e, "nauticle_position_loss");
}

nauticle_status nauticle_check(void* ws, size_t ws_bytes, hipStream_t stream)
{
    size_t err_off;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_plans.find(ws);
        if (it == g_plans.end()) return fail(NAUTICLE_ERR_WORKSPACE, "workspace was not prepared");
        if (ws_bytes < it->second.plan.L.total) return fail(NAUTICLE_ERR_WORKSPACE, "workspace too small");
        err_off = it->second.plan.L.err;
    }
    uint32_t word = 0;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&word, at<char>(ws, err_off), sizeof(word), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(at<char>(ws, err_off), 0, sizeof(word));
    if (e != hipSuccess) return hip_fail(e, "nauticle_check");
    if (word & kErrNonFinite) return fail(NAUTICLE_ERR_NONFINITE, "a non-finite value was produced or given");
    if (word & kErrOverflow) return fail(NAUTICLE_ERR_NEIGHBOUR_OVERFLOW, "a particle had more than max_nbr neighbours");
    if (word & kErrOutOfDomain) return fail(NAUTICLE_ERR_OUT_OF_DOMAIN, "a position lies beyond 2^23 cells");
    if (word & kErrAttribute) return fail(NAUTICLE_ERR_ATTRIBUTE, "a pair-law attribute is out of range");
    return NAUTICLE_OK;
}

const char* nauticle_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
