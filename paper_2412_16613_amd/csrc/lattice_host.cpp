// Lattice (compartment) networks and ensembles: integer form, device layout
// and the schedule/event launches of an advance.  The public entry points in
// host.cpp dispatch here for networks created with lx, ly > 0.

#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include "bwg.h"
#include "bwg_internal.h"
#include "host_internal.h"

namespace bwg {

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// The five Frank reactions of a lattice site, in the order their weights are
// accumulated: A -> L, A -> D, A + L -> 2L, A + D -> 2D, L + D -> 2A.
static const int32_t kFrank[5][2][3] = {
    {{0, 0, 1}, {1, 0, 0}}, {{0, 0, 1}, {0, 1, 0}}, {{1, 0, 1}, {2, 0, 0}},
    {{0, 1, 1}, {0, 2, 0}}, {{1, 1, 0}, {0, 0, 2}},
};

// Integer form of a lattice network: the well-mixed weight rule applied to
// the five site reactions and to the hop rate d (per molecule and
// direction); the site bound 2^B_r covers the weight sum of every site state
// with at most T = 2^P - 1 molecules; a reaction component per site weighs
// 2^B_r, a hop component per (site, direction) (T + 1) c_hop.
int lat_net_setup(bwg_net *n, const bwg_net_desc *d)
{
    if (d->lx < 1 || d->ly < 1) return fail(BWG_EINVAL, "lattice sides must be >= 1");
    if ((int64_t)d->lx * d->ly > LAT_MAX_SITES)
        return fail(BWG_ERANGE, "lattice of %d x %d sites exceeds %d sites", d->lx, d->ly,
                    LAT_MAX_SITES);
    if (n->S != 3 || n->R != 5)
        return fail(BWG_EUNSUPPORTED, "lattices implement the five-reaction Frank table");
    for (int j = 0; j < 5; ++j)
        if (memcmp(&n->reac[3 * j], kFrank[j][0], sizeof kFrank[j][0]) ||
            memcmp(&n->prod[3 * j], kFrank[j][1], sizeof kFrank[j][1]))
            return fail(BWG_EUNSUPPORTED,
                        "lattice reaction %d is not in the order A->L, A->D, A+L->2L, A+D->2D, "
                        "L+D->2A", j);
    if (!d->hop_rates) return fail(BWG_EINVAL, "lattice without hop rates");
    const double hop = d->hop_rates[0];
    for (int x = 0; x < 3; ++x) {
        if (!(d->hop_rates[x] >= 0) || std::isinf(d->hop_rates[x]))
            return fail(BWG_EINVAL, "hop rate must be finite and >= 0");
        if (d->hop_rates[x] != hop)
            return fail(BWG_EUNSUPPORTED, "lattices implement one hop rate for every species");
    }
    const int P = d->site_planes;
    if (P < 1 || P > 8) return fail(BWG_ERANGE, "site_planes %d not in 1..8", P);
    if (d->flags & BWG_EXACT_INTEGER)
        return fail(BWG_EUNSUPPORTED, "lattices take mass-action rates");
    const int prec = d->precision_bits > 0 ? d->precision_bits : 7;

    // scale: s = 2^f / k_ref, the first f at which every positive rate
    // (hops included) has an integral product or one of at least 2^prec
    double k_bi = 0, k_any = hop > 0 ? hop : 0;
    for (int j = 0; j < 5; ++j)
        if (n->rates[j] > 0) {
            k_any = std::max(k_any, n->rates[j]);
            if (j >= 2) k_bi = std::max(k_bi, n->rates[j]);
        }
    if (k_any <= 0) return fail(BWG_EINVAL, "every rate is zero");
    const double k_ref = k_bi > 0 ? k_bi : k_any;
    int f = 0;
    for (; f < 63; ++f) {
        const double s = std::ldexp(1.0, f) / k_ref;
        bool ok = true;
        for (int j = 0; j <= 5 && ok; ++j) {
            const double k = j < 5 ? n->rates[j] : hop;
            if (!(k > 0)) continue;
            const double x = k * s, c = std::nearbyint(x);
            if (!(x == c || c >= std::ldexp(1.0, prec))) ok = false;
        }
        if (ok) break;
    }
    if (f >= 63) return fail(BWG_ERANGE, "no scale reaches %d bits of rate precision", prec);
    bwg_qnet &q = n->q;
    q.f = f;
    q.s = std::ldexp(1.0, f) / k_ref;
    for (int j = 0; j <= 5; ++j) {
        const double c = std::nearbyint((j < 5 ? n->rates[j] : hop) * q.s);
        if (c >= 4294967296.0) return fail(BWG_ERANGE, "weight %d beyond 32 bits", j);
        if (j < 5)
            n->c_lat[j] = q.c[j] = (int64_t)c;
        else
            n->c_hop = (int64_t)c;
    }
    const int64_t T = (1ll << P) - 1;
    int64_t best = 0;
    const int64_t *c = n->c_lat;
    for (int64_t a = 0; a <= T; ++a)
        for (int64_t l = 0; l <= T - a; ++l)
            for (int64_t r = 0; r <= T - a - l; ++r) {
                const int64_t w = (c[0] + c[1]) * a + c[2] * a * l + c[3] * a * r + c[4] * l * r;
                best = std::max(best, w);
            }
    int B = 1;
    while (B < 62 && (1ll << B) < best) ++B;
    LatShape &sh = n->lsh;
    sh.lx = d->lx;
    sh.ly = d->ly;
    sh.S = d->lx * d->ly;
    sh.P = P;
    sh.B_r = B;
    sh.cu = (uint64_t)c[0];
    sh.ca = (uint64_t)c[2];
    sh.ci = (uint64_t)c[4];
    int wx = 1;
    while (wx < 63 && (sh.cu * (uint64_t)T) >> wx) ++wx;
    sh.wx = wx;
    sh.W_R = 1ull << B;
    sh.W_H = (uint64_t)(T + 1) * (uint64_t)n->c_hop;
    sh.Wsite = sh.W_R + 4 * sh.W_H;
    const unsigned __int128 C = (unsigned __int128)sh.S * sh.Wsite;
    if (C >= ((unsigned __int128)1 << 56))
        return fail(BWG_ERANGE, "total component weight beyond 2^56");
    sh.C = (uint64_t)C;
    sh.thresh = (0 - sh.C) % sh.C;
    n->T = (int32_t)T;
    n->lat = true;
    q.B = B;
    q.b = P;
    q.max_total = best;
    q.lambda = (double)sh.C / q.s;
    n->lat_gpu = c[0] == c[1] && c[2] == c[3];
    q.gpu_ok = 0;
    if (n->lat_gpu)
        for (int i = 0; i < kLatVariantCount; ++i)
            if (kLatVariants[i].P == P && kLatVariants[i].bc >= B + 1) q.gpu_ok = 1;
    return BWG_OK;
}

// Words per workgroup slice: 8 once there are enough slices to fill the
// chip (coalesced site records), else one word per workgroup.
static int lat_slice_words(uint64_t M)
{
    const uint64_t words = (M + 31) / 32;
    return words >= 512 ? 4 : 1;
}

// Groups per event launch: at most one workgroup per CU (256), and a band's
// site planes within 224 MB, so that between two visits of a site the planes
// stay in the 256 MB last-level cache instead of going to HBM; bands of
// equal size.
static uint32_t lat_band_groups(const bwg_net *n, int ws, uint64_t groups)
{
    if (ws == 1) return (uint32_t)groups;     // one word per workgroup: no banding
    const uint64_t per_group = (uint64_t)LAT_GROUP_WORDS * n->lsh.S * 3 * n->lsh.P * 4;
    const uint64_t by_cus = 256 / (uint64_t)(LAT_GROUP_WORDS / ws);
    const uint64_t by_cache = (224ull << 20) / per_group;
    const uint64_t b = std::max<uint64_t>(1, std::min(by_cus, by_cache));
    const uint64_t bands = (groups + b - 1) / b;
    return (uint32_t)((groups + bands - 1) / bands);
}

// The event kernel of a lattice for the slice width lat_slice_words picks:
// the LDS-staged one where one exists and staging is asked for, else the
// memory one; compile-time weights before run-time ones, then the fewest
// threshold planes.
static const LatVariant *pick_lat_variant(const bwg_net *n, uint64_t M, bool stage)
{
    if (!n->lat_gpu) return nullptr;
    const LatShape &sh = n->lsh;
    const LatVariant *best = nullptr;
    for (int pass = stage ? 0 : 1; pass < 2 && !best; ++pass)
    for (int i = 0; i < kLatVariantCount; ++i) {
        const LatVariant &v = kLatVariants[i];
        const int ws = lat_slice_words(M);
        if ((v.stage > 0) != (pass == 0)) continue;
        if (v.P != sh.P || v.bc < sh.B_r + 1 || v.ws != ws) continue;
        if (v.cu >= 0 && ((uint64_t)v.cu != sh.cu || (uint64_t)v.ca != sh.ca ||
                          (uint64_t)v.ci != sh.ci))
            continue;
        if (!best) {
            best = &v;
            continue;
        }
        const bool vc = v.cu >= 0, bc = best->cu >= 0;
        if (vc != bc) {
            if (vc) best = &v;
            continue;
        }
        if (v.bc < best->bc) best = &v;
    }
    return best;
}

struct LatLayout {
    uint64_t planes, E, Et, real, blocked, tot, sites, table, scratch, sched, total;
};

static LatLayout lat_layout(const bwg_net *n, uint64_t M, uint64_t table_cap)
{
    const LatShape &sh = n->lsh;
    const uint64_t words = (M + 31) / 32;
    const uint64_t groups = (words + LAT_GROUP_WORDS - 1) / LAT_GROUP_WORDS;
    const uint64_t mp = 32 * words;
    LatLayout L{};
    uint64_t off = 0;
    L.planes = off;
    off = align256(off + groups * LAT_GROUP_WORDS * (uint64_t)sh.S * 3 * sh.P * 4);
    L.E = off;
    off = align256(off + mp * 8);
    L.Et = off;
    off = align256(off + mp * 8);
    L.real = off;
    off = align256(off + words * 8);
    L.blocked = off;
    off = align256(off + words * 8);
    L.tot = off;
    off = align256(off + mp * 3 * 4);
    L.sites = off;
    off = align256(off + (uint64_t)sh.S * 3 * 4);
    L.table = off;
    off = align256(off + table_cap * 8);
    L.scratch = off;
    off = align256(off + 64 * 8);
    L.sched = off;
    off = align256(off + groups * LAT_NCB * (uint64_t)LAT_SLOT * 4);
    L.total = off;
    return L;
}

int lat_state_bytes(const bwg_net *n, uint64_t M, uint64_t table_cap, uint64_t *bytes)
{
    if (!pick_lat_variant(n, M, false))
        return fail(BWG_EUNSUPPORTED, "no lattice event kernel for P=%d, B_r=%d and these weights",
                    n->lsh.P, n->lsh.B_r);
    *bytes = lat_layout(n, M, table_cap).total;
    return BWG_OK;
}

int lat_bind(bwg_ens *e)
{
    const bwg_net *n = e->net;
    e->lvar = pick_lat_variant(n, e->M, e->lat_stage);
    const LatLayout L = lat_layout(n, e->M, e->table_cap);
    e->lat = true;
    e->words = (e->M + 31) / 32;
    e->groups = (e->words + LAT_GROUP_WORDS - 1) / LAT_GROUP_WORDS;
    e->wp = e->words;
    e->nb = n->lsh.P;
    e->planes = (uint32_t *)(e->buf + L.planes);
    e->E = (uint64_t *)(e->buf + L.E);
    e->Et = (uint64_t *)(e->buf + L.Et);
    e->real = (uint64_t *)(e->buf + L.real);
    e->blocked = (uint64_t *)(e->buf + L.blocked);
    e->tot = (int32_t *)(e->buf + L.tot);
    e->sites_dev = (int32_t *)(e->buf + L.sites);
    e->table = (uint64_t *)(e->buf + L.table);
    e->scratch = (uint64_t *)(e->buf + L.scratch);
    e->adv_dev = e->scratch + 8;
    e->sched = (uint32_t *)(e->buf + L.sched);
    return BWG_OK;
}

int lat_init(bwg_ens *e, int32_t mode, const int32_t *counts, hipStream_t s)
{
    const bwg_net *n = e->net;
    const LatShape &sh = n->lsh;
    const int32_t T = n->T;
    int32_t c3[3] = {0, 0, 0};
    if (mode == BWG_INIT_FIXED) {
        if (!counts) return fail(BWG_EINVAL, "fixed init needs the site counts");
        int32_t t = 0;
        for (int x = 0; x < 3; ++x) {
            if (counts[x] < 0) return fail(BWG_EINVAL, "negative initial count");
            c3[x] = counts[x];
            t += counts[x];
        }
        if (t > T) return fail(BWG_ERANGE, "site total %d exceeds the capacity %d", t, T);
        HIP_TRY(launch_lat_init(e->planes, e->words, e->M, sh.S, sh.P, 0, nullptr, c3, 0, 0,
                                e->seed, e->net_id, e->E, e->Et, e->real, e->blocked, s));
    } else if (mode == BWG_INIT_SITES) {
        if (!counts) return fail(BWG_EINVAL, "site init needs the lattice state");
        for (int k = 0; k < sh.S; ++k) {
            int32_t t = 0;
            for (int x = 0; x < 3; ++x) {
                if (counts[3 * k + x] < 0) return fail(BWG_EINVAL, "negative initial count");
                t += counts[3 * k + x];
            }
            if (t > T) return fail(BWG_ERANGE, "site %d total %d exceeds the capacity %d", k, t, T);
        }
        HIP_TRY(hipMemcpyAsync(e->sites_dev, counts, (size_t)sh.S * 3 * 4, hipMemcpyHostToDevice,
                               s));
        HIP_TRY(launch_lat_init(e->planes, e->words, e->M, sh.S, sh.P, 0, e->sites_dev, c3, 0, 0,
                                e->seed, e->net_id, e->E, e->Et, e->real, e->blocked, s));
    } else if (mode == BWG_INIT_UNIFORM_SITE) {
        if (!counts) return fail(BWG_EINVAL, "uniform site init needs lo, hi");
        const int32_t lo = counts[0], hi = counts[1];
        if (lo < 0 || hi < lo) return fail(BWG_EINVAL, "need 0 <= lo <= hi");
        if (hi > T) return fail(BWG_ERANGE, "hi %d exceeds the site capacity %d", hi, T);
        HIP_TRY(launch_lat_init(e->planes, e->words, e->M, sh.S, sh.P, 1, nullptr, c3, lo, hi,
                                e->seed, e->net_id, e->E, e->Et, e->real, e->blocked, s));
    } else {
        return fail(BWG_EINVAL, "init mode %d is not available on a lattice", mode);
    }
    HIP_TRY(launch_fill_u64(e->adv_dev, 1, 0, s));
    e->t_now = 0;
    e->adv = 0;
    e->pending = 0;
    e->emin = e->emax = 0;
    e->base = e->n_chunks = e->cursor = 0;
    e->inited = true;
    return BWG_OK;
}

// Chunk window of an advance whose budgets lie in [kmin, kmax].
static void lat_window(bwg_ens *e, uint64_t kmin, uint64_t kmax)
{
    e->base = e->emin;
    const uint64_t span = e->emax + kmax - e->emin;
    e->n_chunks = (span + LAT_CH - 1) / LAT_CH;
    e->cursor = 0;
    e->emin += kmin;
    e->emax += kmax;
    e->pending = e->n_chunks * (uint64_t)LAT_CH;
}

int lat_schedule(bwg_ens *e, double t_end, hipStream_t s)
{
    if (e->cursor < e->n_chunks)
        return fail(BWG_EINVAL, "the previous advance of this lattice still has pending events");
    uint64_t kmin, kmax;
    int rc = schedule_ensemble(e, t_end, s, &kmin, &kmax);
    if (rc) return rc;
    lat_window(e, kmin, kmax);
    return BWG_OK;
}

int lat_step_schedule(bwg_ens *e, uint64_t n_events, hipStream_t s)
{
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    if (e->cursor < e->n_chunks)
        return fail(BWG_EINVAL, "the previous advance of this lattice still has pending events");
    HIP_TRY(launch_budget(nullptr, 0, 0, n_events, 0, e->seed, e->net_id, e->adv_dev, e->M, e->E,
                          e->Et, s));
    lat_window(e, n_events, n_events);
    return BWG_OK;
}

// Schedule and run the next chunks of the advance, LAT_NCB per pass; at the
// end of the advance every replica's event count moves to its target.
int lat_run(bwg_ens *e, uint64_t max_events, hipStream_t s)
{
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    const bwg_net *n = e->net;
    uint64_t todo = e->n_chunks - e->cursor;
    if (max_events) todo = std::min(todo, (max_events + LAT_CH - 1) / LAT_CH);
    LatArgs a{};
    a.planes = e->planes;
    a.E = e->E;
    a.Et = e->Et;
    a.real = e->real;
    a.blocked = e->blocked;
    a.sched = e->sched;
    a.M = e->M;
    a.seed = e->seed;
    a.base = e->base;
    a.net_id = e->net_id;
    a.sh = n->lsh;
    const uint32_t band = lat_band_groups(n, e->lvar->ws, e->groups);
    while (todo) {
        const uint32_t nc = (uint32_t)std::min<uint64_t>(todo, LAT_NCB);
        a.chunk0 = (uint32_t)e->cursor;
        a.n_chunks = nc;
        HIP_TRY(launch_lat_schedule(a, (uint32_t)e->groups, s));
        for (uint64_t g0 = 0; g0 < e->groups; g0 += band) {
            a.g0 = (uint32_t)g0;
            a.ng = (uint32_t)std::min<uint64_t>(band, e->groups - g0);
            hipEvent_t ev = nullptr;
            int rc = mark_begin(e, s, &ev);
            if (rc) return rc;
            HIP_TRY(e->lvar->fn(a, e->words, s));
            rc = mark_end(e, s, ev);
            if (rc) return rc;
        }
        e->cursor += nc;
        todo -= nc;
    }
    if (e->cursor == e->n_chunks && e->pending) {
        HIP_TRY(launch_copy_u64(e->Et, e->E, 32 * e->words, s));
    }
    e->pending = (e->n_chunks - e->cursor) * (uint64_t)LAT_CH;
    return BWG_OK;
}

int lat_read_counts(bwg_ens *e, int32_t *dst, hipStream_t s)
{
    HIP_TRY(launch_lat_totals(e->planes, e->M, e->net->lsh.S, e->net->lsh.P, dst, s));
    return BWG_OK;
}

int lat_histogram(bwg_ens *e, int32_t n_bins, uint64_t *dst, hipStream_t s)
{
    HIP_TRY(launch_lat_totals(e->planes, e->M, e->net->lsh.S, e->net->lsh.P, e->tot, s));
    HIP_TRY(launch_lat_histogram(e->tot, e->M, n_bins, dst, s));
    return BWG_OK;
}

}  // namespace bwg

using namespace bwg;

static_assert(LAT_CH == BWG_LAT_CHUNK_EVENTS && LAT_NCB == BWG_LAT_PASS_CHUNKS,
              "the schedule geometry include/bwg.h states");

extern "C" int bwg_net_lattice(const bwg_net *n, bwg_lattice_info *out)
{
    if (!n || !out) return fail(BWG_EINVAL, "null argument");
    if (!n->lat) return fail(BWG_EINVAL, "not a lattice network");
    const LatShape &sh = n->lsh;
    out->lx = sh.lx;
    out->ly = sh.ly;
    out->sites = sh.S;
    out->P = sh.P;
    out->T = n->T;
    out->B_r = sh.B_r;
    out->c_hop = n->c_hop;
    out->C = sh.C;
    out->max_site = n->q.max_total;
    out->s = n->q.s;
    out->lambda = n->q.lambda;
    return BWG_OK;
}

extern "C" int bwg_ensemble_read_sites(bwg_ens *e, uint64_t first, uint64_t count,
                                       int32_t *dev_dst, void *stream)
{
    TraceRange trace_("bwg_ensemble_read_sites");
    if (!e || !dev_dst) return fail(BWG_EINVAL, "null argument");
    if (!e->lat) return fail(BWG_EINVAL, "not a lattice ensemble");
    if (first > e->M || count > e->M - first) return fail(BWG_EINVAL, "replica range out of bounds");
    if (!count) return BWG_OK;
    HIP_TRY(launch_lat_sites(e->planes, e->net->lsh.S, e->net->lsh.P, first, count, dev_dst,
                             (hipStream_t)stream));
    return BWG_OK;
}

extern "C" int bwg_ensemble_read_blocked(bwg_ens *e, uint64_t *dev_dst, void *stream)
{
    if (!e || !dev_dst) return fail(BWG_EINVAL, "null argument");
    if (!e->lat) return fail(BWG_EINVAL, "not a lattice ensemble");
    HIP_TRY(launch_copy_u64(e->blocked, dev_dst, e->words, (hipStream_t)stream));
    return BWG_OK;
}
