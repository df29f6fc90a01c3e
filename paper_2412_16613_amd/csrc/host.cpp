// C ABI of the bit-parallel Gillespie library: networks, quantisation,
// ensembles, launches.  See include/bwg.h for the contract of every call.

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bwg.h"
#include "bwg_internal.h"
#include "host_internal.h"

namespace bwg {
int poisson_table_q(double mu, int64_t *k_lo, std::vector<uint64_t> &T);
}

using namespace bwg;

// ---- errors ------------------------------------------------------------------

namespace bwg {
static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace bwg

extern "C" const char *bwg_last_error(void) { return g_err.c_str(); }

// ---- networks ------------------------------------------------------------------

static int64_t comb_h(const int32_t *r, const int64_t *N, int S)
{
    int64_t v = 1;
    for (int x = 0; x < S; ++x) {
        if (r[x] == 1)
            v *= N[x];
        else if (r[x] == 2)
            v *= N[x] * (N[x] - 1) / 2;
    }
    return v;
}

// Total weight sum_j c_j h_j(N) of the 3-species state (a, b, c).
static int64_t total_weight_at(const bwg_net &n, int64_t a, int64_t b, int64_t c)
{
    const int64_t st[3] = {a, b, c};
    int64_t t = 0;
    for (int j = 0; j < n.R; ++j)
        if (n.q.c[j]) t += n.q.c[j] * comb_h(&n.reac[j * 3], st, 3);
    return t;
}

// Smallest and largest total weight over every state with n_tot molecules
// (3 species), exactly and in O(n_tot): with the first count a fixed, every
// h_j is a polynomial of degree at most 2 in the second count t (the third
// is n_tot - a - t), so the total is an integer quadratic W(t) on [0, M],
// M = n_tot - a.  Its extremes over the integers lie at the ends of the range
// or at the integers next to the vertex t* = 1/2 - (W(1) - W(0)) / d2, d2 =
// W(2) - 2 W(1) + W(0) (the maximum there when d2 < 0, the minimum when
// d2 > 0); every candidate is evaluated exactly in int64, and the window
// around t* is wide enough for the rounding of t* in binary64.
static void total_weight_range(const bwg_net &n, int64_t *lo, int64_t *hi)
{
    int64_t best = 0, least = INT64_MAX;
    const int64_t N = n.n_tot;
    for (int64_t a = 0; a <= N; ++a) {
        const int64_t M = N - a;
        auto take = [&](int64_t t) {
            if (t < 0 || t > M) return;
            const int64_t v = total_weight_at(n, a, t, M - t);
            if (v > best) best = v;
            if (v < least) least = v;
        };
        take(0);
        take(M);
        if (M < 2) continue;
        const int64_t w0 = total_weight_at(n, a, 0, M), w1 = total_weight_at(n, a, 1, M - 1),
                      w2 = total_weight_at(n, a, 2, M - 2);
        const int64_t d2 = w2 - 2 * w1 + w0;
        if (d2 == 0) continue;  // linear in t: the ends
        const double ts = 0.5 - (double)(w1 - w0) / (double)d2;
        if (!(ts > -2.0 && ts < (double)M + 2.0)) continue;
        const int64_t f = (int64_t)std::floor(ts);
        for (int64_t t = f - 1; t <= f + 2; ++t) take(t);
    }
    *lo = least;
    *hi = best;
}

// Bound of the total weight for every network but the 3-species closed
// ones: sum_j c_j max h_j, each reaction's largest factor over the state
// space -- the simplex of n_tot molecules (N_X: n, N_X N_Y: floor(n/2)
// ceil(n/2), N_X (N_X - 1) / 2: n (n - 1) / 2) or, for an open network, the
// box of counts at most n_tot (n, n^2, n (n - 1) / 2: the corner).  Returns
// false if the bound passes 2^62.
static bool total_weight_bound(const bwg_net &n, int64_t *hi)
{
    const __int128 N = n.n_tot;
    __int128 t = 0;
    for (int j = 0; j < n.R; ++j) {
        int xs[2], k = 0;
        for (int x = 0; x < n.S; ++x)
            for (int m = 0; m < n.reac[j * n.S + x]; ++m) xs[k++] = x;
        __int128 h;
        if (k == 1)
            h = N;
        else if (xs[0] != xs[1])
            h = n.open ? N * N : (N / 2) * (N - N / 2);
        else
            h = N * (N - 1) / 2;
        t += (__int128)n.q.c[j] * h;
        if (t > ((__int128)1 << 62)) return false;
    }
    *hi = (int64_t)t;
    return true;
}

static int ilog2_exact(int64_t c)  // log2 of a power of two, else -2
{
    if (c <= 0 || (c & (c - 1))) return -2;
    int k = 0;
    while ((1ll << k) < c) ++k;
    return k;
}

// Frank-family recognition for the bit-sliced kernel (species L, D, A).
static void classify(bwg_net &n)
{
    n.shape_ok = false;
    if (n.S != 3 || n.open) return;
    static const int32_t RX[5][2][3] = {
        {{0, 0, 1}, {1, 0, 0}},  // A -> L
        {{0, 0, 1}, {0, 1, 0}},  // A -> D
        {{1, 0, 1}, {2, 0, 0}},  // A + L -> 2L
        {{0, 1, 1}, {0, 2, 0}},  // A + D -> 2D
        {{1, 1, 0}, {0, 0, 2}},  // L + D -> 2A
    };
    int64_t c[5] = {0, 0, 0, 0, 0};
    int last = -1;
    bool ghosts_started = false;
    for (int j = 0; j < n.R; ++j) {
        const int32_t *r = &n.reac[j * 3], *p = &n.prod[j * 3];
        const bool ghost = r[0] == p[0] && r[1] == p[1] && r[2] == p[2];
        if (ghost) {
            ghosts_started = true;
            continue;
        }
        if (ghosts_started) return;
        int t = -1;
        for (int k = 0; k < 5; ++k)
            if (!memcmp(r, RX[k][0], sizeof(RX[k][0])) && !memcmp(p, RX[k][1], sizeof(RX[k][1])))
                t = k;
        if (t < 0 || t <= last) return;
        last = t;
        c[t] = n.q.c[j];
    }
    if (c[0] != c[1]) return;
    if (c[2] != c[3]) return;
    if (c[0] >= (1ll << 32)) return;
    const int fa = c[2] ? ilog2_exact(c[2]) : -1;
    const int fi = c[4] ? ilog2_exact(c[4]) : -1;
    if (fa == -2 || fi == -2) return;
    n.shape.cu = (uint32_t)c[0];
    n.shape.fa = fa;
    n.shape.fi = fi;
    n.shape_ok = true;
}

static void classify_plain(bwg_net &n)
{
    n.plain_ok = false;
    if (n.S != 3 || n.open || n.R > 16) return;
    for (int j = 0; j < n.R; ++j) {
        const int32_t *r = &n.reac[j * 3], *p = &n.prod[j * 3];
        PlainReaction &rx = n.prx[j];
        int xs[2], k = 0;
        for (int x = 0; x < 3; ++x)
            for (int m = 0; m < r[x]; ++m) xs[k++] = x;
        if (k == 1) {
            rx.kind = 0;
            rx.x = rx.y = xs[0];
        } else if (xs[0] != xs[1]) {
            rx.kind = 1;
            rx.x = xs[0];
            rx.y = xs[1];
        } else {
            rx.kind = 2;
            rx.x = rx.y = xs[0];
        }
        for (int x = 0; x < 3; ++x) rx.d[x] = p[x] - r[x];
        if (n.q.c[j] >= (1ll << 32)) return;
        rx.c = (uint32_t)n.q.c[j];
    }
    n.plain_ok = true;
}

// Reaction table of the general bit-sliced kernel: the weight kind of each
// reaction (N_X; N_L N_D, N_L N_A, N_D N_A; N_X (N_X - 1) / 2), its integer
// weight and state change.
// Networks of other than 3 species and open networks: the compiled general
// kernel takes any such table whose weights fit 32 bits and whose changes
// are in {-2..2} per species.
static void classify_wide(bwg_net &n)
{
    n.wide_ok = false;
    if (!n.wide || n.R > bwg::kGenMaxR) return;
    for (int j = 0; j < n.R; ++j) {
        if (n.q.c[j] >= (1ll << 32)) return;
        for (int x = 0; x < n.S; ++x) {
            const int dv = n.prod[j * n.S + x] - n.reac[j * n.S + x];
            if (dv < -2 || dv > 2) return;
        }
    }
    n.wide_ok = true;
}

static void classify_generic(bwg_net &n)
{
    n.gen_ok = false;
    if (n.S != 3 || n.open || n.R > bwg::kGenMaxR) return;
    bwg::GenNet &g = n.gen;
    g = bwg::GenNet{};
    g.R = n.R;
    for (int j = 0; j < n.R; ++j) {
        const int32_t *r = &n.reac[j * 3], *p = &n.prod[j * 3];
        int xs[2], k = 0;
        for (int x = 0; x < 3; ++x)
            for (int m = 0; m < r[x]; ++m) xs[k++] = x;
        int kind;
        if (k == 1)
            kind = xs[0];
        else if (xs[0] == xs[1])
            kind = 6 + xs[0];
        else
            kind = xs[0] == 0 ? (xs[1] == 1 ? 3 : 4) : 5;
        if (n.q.c[j] >= (1ll << 32)) return;
        g.c[j] = (uint32_t)n.q.c[j];
        g.kind[j] = (uint8_t)kind;
        if (g.c[j]) g.used |= 1u << kind;
        for (int x = 0; x < 3; ++x) {
            g.d[j][x] = (int8_t)(p[x] - r[x]);
            if (p[x] != r[x]) g.change |= 1u << j;
        }
    }
    for (int k = 0; k < 9; ++k)
        if ((g.used >> k) & 1u) g.slot[k] = (uint8_t)g.n_slots++;
    n.gen_ok = true;
}

extern "C" int bwg_net_create(const bwg_net_desc *d, bwg_net **out)
{
    TraceRange trace_("bwg_net_create");
    if (!d || !out) return fail(BWG_EINVAL, "null argument");
    *out = nullptr;
    const int S = d->n_species, R = d->n_reactions;
    if (S < 1 || S > BWG_MAX_SPECIES) return fail(BWG_EINVAL, "n_species %d out of range", S);
    if (R < 1 || R > BWG_MAX_REACTIONS) return fail(BWG_EINVAL, "n_reactions %d out of range", R);
    if (!d->reactants || !d->products || !d->rates) return fail(BWG_EINVAL, "null table");
    if (d->n_tot < 1) return fail(BWG_EINVAL, "n_tot must be >= 1");
    const bool lattice = d->lx || d->ly;
    const bool open_net = (d->flags & BWG_OPEN) != 0;
    if (lattice && (S != 3 || open_net))
        return fail(BWG_EUNSUPPORTED, "lattices are closed networks of 3 species");
    if (!lattice && d->n_tot >= (1ll << 14)) return fail(BWG_ERANGE, "n_tot beyond 14 count planes");
    auto n = new bwg_net();
    n->S = S;
    n->open = open_net;
    n->wide = S != 3 || open_net;
    n->R = R;
    n->reac.assign(d->reactants, d->reactants + S * R);
    n->prod.assign(d->products, d->products + S * R);
    n->rates.assign(d->rates, d->rates + R);
    n->n_tot = d->n_tot;
    for (int j = 0; j < R; ++j) {
        int o = 0, op = 0;
        for (int x = 0; x < S; ++x) {
            const int32_t r = n->reac[j * S + x], p = n->prod[j * S + x];
            if (r < 0 || p < 0) {
                delete n;
                return fail(BWG_EINVAL, "reaction %d: negative stoichiometry", j);
            }
            o += r;
            op += p;
        }
        if (o < 1 || o > 2) {
            delete n;
            return fail(BWG_EINVAL, "reaction %d: order %d not in {1, 2}", j, o);
        }
        if (o != op && !open_net) {
            delete n;
            return fail(BWG_EINVAL, "reaction %d does not conserve the molecule count", j);
        }
        const double k = n->rates[j];
        if (!(k >= 0) || std::isinf(k)) {
            delete n;
            return fail(BWG_EINVAL, "reaction %d: rate must be finite and >= 0", j);
        }
    }
    n->q.n_species = S;
    n->q.n_reactions = R;
    if (lattice) {
        n->lx = d->lx;
        n->ly = d->ly;
        const int rc = lat_net_setup(n, d);
        if (rc) {
            delete n;
            return rc;
        }
        *out = n;
        return BWG_OK;
    }
    // ---- quantisation: integer weights c_j = rint(k_j s), s = 2^f / k_ref
    bwg_qnet &q = n->q;
    const int prec = d->precision_bits > 0 ? d->precision_bits : 7;
    if (d->flags & BWG_EXACT_INTEGER) {
        for (int j = 0; j < R; ++j) {
            const double k = n->rates[j];
            if (k != std::floor(k) || k >= 4294967296.0) {
                delete n;
                return fail(BWG_EINVAL, "exact-integer table: rate %d is not a 32-bit integer", j);
            }
            q.c[j] = (int64_t)k;
        }
        q.f = 0;
        q.s = 1.0;
    } else {
        double k_bi = 0, k_any = 0;
        for (int j = 0; j < R; ++j) {
            int o = 0;
            for (int x = 0; x < S; ++x) o += n->reac[j * S + x];
            if (n->rates[j] > 0) {
                k_any = std::max(k_any, n->rates[j]);
                if (o == 2) k_bi = std::max(k_bi, n->rates[j]);
            }
        }
        if (k_any <= 0) {
            delete n;
            return fail(BWG_EINVAL, "every rate is zero");
        }
        const double k_ref = k_bi > 0 ? k_bi : k_any;
        int f = 0;
        for (; f < 63; ++f) {
            const double s = std::ldexp(1.0, f) / k_ref;
            bool ok = true;
            for (int j = 0; j < R && ok; ++j) {
                if (!(n->rates[j] > 0)) continue;
                const double x = n->rates[j] * s;
                const double c = std::nearbyint(x);
                if (!(x == c || c >= std::ldexp(1.0, prec))) ok = false;
            }
            if (ok) break;
        }
        if (f >= 63) {
            delete n;
            return fail(BWG_ERANGE, "no scale reaches %d bits of rate precision", prec);
        }
        q.f = f;
        q.s = std::ldexp(1.0, f) / k_ref;
        for (int j = 0; j < R; ++j) {
            const double c = std::nearbyint(n->rates[j] * q.s);
            if (c >= 4294967296.0) {
                delete n;
                return fail(BWG_ERANGE, "weight of reaction %d beyond 32 bits", j);
            }
            q.c[j] = (int64_t)c;
        }
    }
    int64_t min_total = -1;
    if (n->wide) {
        if (!total_weight_bound(*n, &q.max_total)) {
            delete n;
            return fail(BWG_ERANGE, "total weight beyond %d threshold planes", kMaxThresholdPlanes);
        }
    } else {
        total_weight_range(*n, &min_total, &q.max_total);
    }
    int B = 1;
    while (B < 63 && (1ll << B) < q.max_total) ++B;
    if (B + (q.max_total == (1ll << B) ? 1 : 0) > kMaxThresholdPlanes) {
        const long long total = (long long)q.max_total;   // q lives in n
        delete n;
        return fail(BWG_ERANGE, "total weight %lld needs %d threshold planes (max %d)", total, B,
                    kMaxThresholdPlanes);
    }
    q.B = B;
    int b = 1;
    while ((1ll << b) <= n->n_tot) ++b;
    q.b = b;
    q.lambda = std::ldexp(1.0, B) / q.s;
    // shared-threshold range: the total weight when no state changes it (the
    // ghost reactions of Eq. (9) make it N(N-1)/2), else 2^B; 0 past 32 bits
    const int64_t z = (min_total == q.max_total && q.max_total > 0) ? q.max_total : (1ll << B);
    q.z_shared = z < (1ll << 32) ? z : 0;
    classify(*n);
    classify_plain(*n);
    classify_generic(*n);
    classify_wide(*n);
    q.gpu_ok = (n->shape_ok || n->gen_ok || n->wide_ok) ? 1 : 0;
    *out = n;
    return BWG_OK;
}

extern "C" int bwg_net_quantized(const bwg_net *n, bwg_qnet *out)
{
    if (!n || !out) return fail(BWG_EINVAL, "null argument");
    *out = n->q;
    return BWG_OK;
}

extern "C" void bwg_net_destroy(bwg_net *n) { delete n; }

extern "C" int bwg_poisson_table(double mu, int64_t *k_lo, uint64_t *table, uint64_t cap,
                                 uint64_t *len)
{
    if (!k_lo || !len) return fail(BWG_EINVAL, "null argument");
    std::vector<uint64_t> T;
    if (poisson_table_q(mu, k_lo, T) != 0) return fail(BWG_EINVAL, "invalid mean %g", mu);
    *len = T.size();
    if (T.size() > cap || !table)
        return table ? fail(BWG_ERANGE, "table needs %zu entries", T.size()) : BWG_OK;
    memcpy(table, T.data(), T.size() * sizeof(uint64_t));
    return BWG_OK;
}

// Cached pinned copy of the table for mean mu.
int bwg::get_table(bwg_net *n, double mu, const Table **out, bool pinned)
{
    uint64_t key;
    memcpy(&key, &mu, sizeof key);
    std::lock_guard<std::mutex> g(n->mu);
    auto it = n->tables.find(key);
    if (it == n->tables.end()) {
        Table t{0, 0, {}, nullptr};
        if (poisson_table_q(mu, &t.k_lo, t.vals) != 0) return fail(BWG_EINVAL, "invalid mean %g", mu);
        t.len = t.vals.size();
        it = n->tables.emplace(key, std::move(t)).first;
    }
    Table &t = it->second;
    if (pinned && !t.host) {
        HIP_TRY(hipHostMalloc((void **)&t.host, t.len * sizeof(uint64_t), hipHostMallocDefault));
        memcpy(t.host, t.vals.data(), t.len * sizeof(uint64_t));
    }
    *out = &t;
    return BWG_OK;
}

// ---- ensembles ------------------------------------------------------------------

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

struct Layout {
    uint64_t wp, planes, counts, E, Et, real, table, scratch, total;
};

static const WmVariant *pick_variant(const bwg_net *n)
{
    if (!n->shape_ok) return nullptr;
    const int b = n->q.b;
    const int need_bc = n->q.B + (n->q.max_total == (1ll << n->q.B) ? 1 : 0);
    const int fa = n->shape.fa, fi = n->shape.fi;
    const int f_common = fa >= 0 ? fa : fi;
    const bool same = (fa < 0 || fi < 0 || fa == fi);
    const WmVariant *best = nullptr;
    for (int i = 0; i < kWmVariantCount; ++i) {
        const WmVariant &v = kWmVariants[i];
        if (v.nb < b || v.bc < need_bc) continue;
        // a variant fixed to one molecule count (exact register widths)
        // serves exactly that count and selection width
        if (v.nt > 0 && (v.nt != n->n_tot || v.bs != need_bc || fa < 0 || fi < 0)) continue;
        if (v.fa >= 0 && !(same && v.fa == f_common && f_common >= 0)) continue;
        if (v.cu >= 0 && (uint32_t)v.cu != n->shape.cu) continue;
        if (fa >= v.bc || fi >= v.bc) continue;
        if (!best) {
            best = &v;
            continue;
        }
        // prefer a compile-time shift, then the fewest planes
        const bool vs = v.fa >= 0, bs = best->fa >= 0;
        if (vs != bs) {
            if (vs) best = &v;
            continue;
        }
        if (v.nb + v.bc < best->nb + best->bc) best = &v;
    }
    return best;
}

static Layout layout(const bwg_net *n, uint64_t M, int engine, uint64_t table_cap,
                     const WmVariant *v)
{
    Layout L{};
    const uint64_t words = (M + 31) / 32;
    L.wp = (words + 63) / 64 * 64;
    const uint64_t mp = 32 * L.wp;
    uint64_t off = 0;
    if (engine != BWG_ENGINE_PLAIN) {
        L.planes = off;
        off = align256(off + (uint64_t)n->S * (uint64_t)n->q.b * L.wp * 4);
        L.counts = ~0ull;
    } else {
        L.counts = off;
        off = align256(off + 3ull * mp * 4);
        L.planes = ~0ull;
    }
    L.E = off;
    off = align256(off + mp * 8);
    L.Et = off;
    off = align256(off + mp * 8);
    L.real = off;
    off = align256(off + (engine != BWG_ENGINE_PLAIN ? L.wp : mp) * 8);
    L.table = off;
    off = align256(off + table_cap * 8);
    L.scratch = off;
    off = align256(off + 64 * 8);
    L.total = off;
    (void)n;
    return L;
}

static const GenVariant *pick_gen_variant(const bwg_net *n)
{
    if (!n->gen_ok) return nullptr;
    const int need_bc = n->q.B + (n->q.max_total == (1ll << n->q.B) ? 1 : 0);
    const GenVariant *best = nullptr;
    for (int i = 0; i < kGenVariantCount; ++i) {
        const GenVariant &v = kGenVariants[i];
        if (v.nb < n->q.b || v.bc < need_bc) continue;
        if (!best || v.nb + v.bc < best->nb + best->bc) best = &v;
    }
    return best;
}

// Kernel of an engine for a network: the Frank-family kernel where it
// applies (unless generic is asked for), else the general bit-sliced one.
// Threshold planes the selection needs: B, or B + 1 when the largest total
// weight is exactly 2^B.
static int need_planes(const bwg_net *n)
{
    return n->q.B + (n->q.max_total == (1ll << n->q.B) ? 1 : 0);
}

// Networks on the general kernels: the precompiled one, else (other species
// counts, open networks, weights beyond 32 threshold planes) only the one
// compiled for the network.
static bool gen_path(const bwg_net *n, int engine, bool generic)
{
    return engine == BWG_ENGINE_BITWISE && (n->wide || generic || !n->shape_ok);
}

// The kernels compiled at run time that an ensemble of n on engine runs,
// given the precompiled variant var: the general one (gen) on the general
// path, and the Frank-family one (frank) for a Frank-family network on a
// run-time weight variant, or on none beyond 32 threshold planes.  The
// Frank one is built at the first launch of the bit-sliced engine (batch
// members never launch alone and never build it); the precompiled variant
// stays for the lanes engine and explicit block sizes.
static void jit_plan(const bwg_net *n, int engine, const WmVariant *var, bool generic,
                     bool jit_ok, bool *gen, bool *frank)
{
    const bool gp = gen_path(n, engine, generic);
    *gen = gp && jit_ok;
    *frank = var ? (jit_ok && (var->fa < 0 || var->cu < 0) && jit_frank_fits(n))
                 : (engine == BWG_ENGINE_BITWISE && !gp && jit_ok && n->shape_ok &&
                    jit_frank_fits(n));
}

// The kernels an engine runs a network on.  Weights beyond 32 threshold
// planes run only the bit-sliced kernels compiled for the network (jit:
// run-time compiles allowed).
static int check_engine(const bwg_net *n, int engine, const WmVariant **v,
                        const GenVariant **gv = nullptr, bool generic = false, bool jit = true)
{
    *v = nullptr;
    if (gv) *gv = nullptr;
    const bool wide_planes = need_planes(n) > 32;
    if (engine == BWG_ENGINE_BITWISE && n->wide) {
        // only the kernel compiled for the network (checked at creation)
        if (!n->wide_ok)
            return fail(BWG_EUNSUPPORTED, "no bit-sliced kernel for this network (changes beyond "
                                          "+-2 or weights beyond 32 bits)");
        return BWG_OK;
    }
    if (engine == BWG_ENGINE_BITWISE && (generic || !n->shape_ok)) {
        const GenVariant *g = wide_planes ? nullptr : pick_gen_variant(n);
        if (!g && !(wide_planes && n->gen_ok && jit))
            return fail(BWG_EUNSUPPORTED,
                        wide_planes ? "weights beyond 32 threshold planes run the kernel compiled "
                                      "for the network (not with BWG_OPT_NO_JIT)"
                                    : "no bit-sliced kernel for this network (b=%d B=%d)",
                        n->q.b, n->q.B);
        if (gv) *gv = g;
        return BWG_OK;
    }
    if (engine == BWG_ENGINE_BITWISE || engine == BWG_ENGINE_LANES) {
        if (!n->shape_ok)
            return fail(BWG_EUNSUPPORTED,
                        "network is not of the Frank family the lanes engine implements");
        *v = pick_variant(n);
        if (!*v && engine == BWG_ENGINE_BITWISE && wide_planes && jit && jit_frank_fits(n))
            return BWG_OK;  // the Frank kernels compiled for the network only
        if (!*v)
            return fail(BWG_EUNSUPPORTED, "no bit-sliced kernel for b=%d B=%d fa=%d fi=%d%s",
                        n->q.b, n->q.B, n->shape.fa, n->shape.fi,
                        wide_planes ? " (beyond 32 threshold planes: the bit-sliced engine's "
                                      "compiled kernels)" : "");
        // the lanes engine compares in 32-bit arithmetic: every cumulative
        // weight must stay below 2^32 (it does whenever a bucket holds the
        // planes; checked here for the record)
        if (engine == BWG_ENGINE_LANES && (n->q.B > 32 || n->q.max_total >= (1ll << 32)))
            return fail(BWG_EUNSUPPORTED, "lanes engine needs total weights below 2^32");
        return BWG_OK;
    }
    if (engine == BWG_ENGINE_PLAIN) {
        if (!n->plain_ok) return fail(BWG_EUNSUPPORTED, "network not supported by the plain engine");
        if (n->q.B > 32)
            return fail(BWG_EUNSUPPORTED, "the plain engine draws 32-bit thresholds (B = %d)",
                        n->q.B);
        return BWG_OK;
    }
    return fail(BWG_EINVAL, "unknown engine %d", engine);
}

extern "C" int bwg_ensemble_state_bytes(const bwg_net *n, uint64_t M, const bwg_opts *o,
                                        uint64_t *bytes)
{
    if (!n || !bytes) return fail(BWG_EINVAL, "null argument");
    if (M == 0 || M >= (1ull << 32)) return fail(BWG_EINVAL, "replica count out of range");
    const int engine = o ? o->engine : BWG_ENGINE_BITWISE;
    const uint64_t cap = (o && o->table_capacity) ? o->table_capacity : 65536;
    if (o && (o->block < 0 || o->block > 256 || o->block % 64))
        return fail(BWG_EINVAL, "block %d: the event kernels take 64, 128, 192 or 256 threads",
                    o->block);
    const bool generic = o && (o->flags & BWG_OPT_GENERIC_KERNEL);
    if (generic && (n->lat || engine != BWG_ENGINE_BITWISE))
        return fail(BWG_EUNSUPPORTED, "the general kernel is a well-mixed bit-sliced engine");
    const uint64_t wb = o ? o->word_bits : 0;
    if (wb != 0 && wb != 16 && wb != 32 && wb != 64)
        return fail(BWG_EINVAL, "word_bits %llu: 16, 32 or 64", (unsigned long long)wb);
    if (wb == 16 || wb == 64) {
        const WmVariant *v = nullptr;
        if (engine != BWG_ENGINE_BITWISE || n->lat || generic || !n->shape_ok ||
            !(v = pick_variant(n)) || v->fa < 0 || v->cu < 0)
            return fail(BWG_EUNSUPPORTED,
                        "%llu-replica words run the precompiled compile-time Frank kernels only",
                        (unsigned long long)wb);
    }
    if (o && (o->flags & BWG_OPT_SHARED_THRESHOLD)) {
        if (n->lat || engine == BWG_ENGINE_PLAIN)
            return fail(BWG_EUNSUPPORTED,
                        "shared thresholds run on the well-mixed bit-plane engines");
        if (generic || !n->shape_ok)
            return fail(BWG_EUNSUPPORTED, "shared thresholds run on Frank-family networks");
        if (!n->q.z_shared)
            return fail(BWG_ERANGE, "shared-threshold range beyond 32 bits");
    }
    if (n->lat) {
        if (engine != BWG_ENGINE_BITWISE)
            return fail(BWG_EUNSUPPORTED, "lattices run on the bit-sliced engine only");
        return lat_state_bytes(n, M, cap, bytes);
    }
    const WmVariant *v;
    const bool jit = !(o && (o->flags & BWG_OPT_NO_JIT));
    int rc = check_engine(n, engine, &v, nullptr, generic, jit);
    if (rc) return rc;
    if (engine == BWG_ENGINE_BITWISE && !v && n->shape_ok && !generic && o && o->block > 0)
        return fail(BWG_EUNSUPPORTED, "beyond 32 threshold planes the compiled kernels choose "
                                      "their block size (block = 0)");
    *bytes = layout(n, M, engine, cap, v).total;
    return BWG_OK;
}

extern "C" int bwg_ensemble_create(const bwg_net *n, uint64_t M, uint64_t seed, uint32_t net_id,
                                   void *dev_buf, uint64_t buf_bytes, const bwg_opts *o,
                                   bwg_ens **out)
{
    TraceRange trace_("bwg_ensemble_create");
    if (!n || !out || !dev_buf) return fail(BWG_EINVAL, "null argument");
    *out = nullptr;
    if ((uintptr_t)dev_buf & 255) return fail(BWG_EINVAL, "device buffer not 256-byte aligned");
    uint64_t need;
    int rc = bwg_ensemble_state_bytes(n, M, o, &need);
    if (rc) return rc;
    if (buf_bytes < need)
        return fail(BWG_ENOMEM, "buffer of %llu bytes, need %llu", (unsigned long long)buf_bytes,
                    (unsigned long long)need);
    auto e = new bwg_ens();
    rc = ens_bind(e, n, M, seed, net_id, dev_buf, buf_bytes, o);
    if (rc) {
        delete e;
        return rc;
    }
    *out = e;
    return BWG_OK;
}

// Fill ensemble e (fresh) for a validated buffer of at least the state bytes.
int bwg::ens_bind(bwg_ens *e, const bwg_net *n, uint64_t M, uint64_t seed, uint32_t net_id,
                  void *dev_buf, uint64_t buf_bytes, const bwg_opts *o)
{
    e->net = const_cast<bwg_net *>(n);
    e->M = M;
    e->seed = seed;
    e->net_id = net_id;
    e->engine = o ? o->engine : BWG_ENGINE_BITWISE;
    e->block = o ? o->block : 0;
    e->table_cap = (o && o->table_capacity) ? o->table_capacity : 65536;
    e->epl = o ? o->events_per_launch : 0;
    e->timed = o && (o->flags & BWG_OPT_TIME_KERNELS);
    e->lat_stage = !(o && (o->flags & BWG_OPT_NO_LDS_STAGE));
    e->word_bits = (o && o->word_bits) ? (int)o->word_bits : 32;
    e->zs = (o && (o->flags & BWG_OPT_SHARED_THRESHOLD)) ? (uint32_t)n->q.z_shared : 0;
    e->buf = (uint8_t *)dev_buf;
    e->bytes = buf_bytes;
    if (n->lat) return lat_bind(e);
    const bool generic = o && (o->flags & BWG_OPT_GENERIC_KERNEL);
    const bool jit_ok = !(o && (o->flags & BWG_OPT_NO_JIT));
    check_engine(n, e->engine, &e->var, &e->gvar, generic, jit_ok);
    if (gen_path(n, e->engine, generic) && !e->gvar && !jit_ok)
        return fail(BWG_EUNSUPPORTED, "this network runs only its compiled kernel (no BWG_OPT_NO_JIT)");
    bool want_gen = false;
    jit_plan(n, e->engine, e->var, generic, jit_ok, &want_gen, &e->want_jit_frank);
    if (want_gen) {
        const int rc = jit_get(const_cast<bwg_net *>(n), &e->jit);
        if (rc) return rc;
    }
    const Layout L = layout(n, M, e->engine, e->table_cap, e->var);
    e->buf = (uint8_t *)dev_buf;
    e->bytes = buf_bytes;
    e->wp = L.wp;
    e->nb = n->q.b;  // planes per species in memory
    if (e->engine != BWG_ENGINE_PLAIN)
        e->planes = (uint32_t *)(e->buf + L.planes);
    else
        e->counts = (int32_t *)(e->buf + L.counts);
    e->E = (uint64_t *)(e->buf + L.E);
    e->Et = (uint64_t *)(e->buf + L.Et);
    e->real = (uint64_t *)(e->buf + L.real);
    e->table = (uint64_t *)(e->buf + L.table);
    e->scratch = (uint64_t *)(e->buf + L.scratch);
    e->adv_dev = e->scratch + 8;
    return BWG_OK;
}

extern "C" void bwg_ensemble_destroy(bwg_ens *e) { delete e; }

extern "C" int bwg_ensemble_set_lanes_words(bwg_ens *e, uint64_t n_words)
{
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (e->lat || e->engine == BWG_ENGINE_PLAIN || !e->net->shape_ok)
        return fail(BWG_EINVAL, "only Frank-family bit-plane ensembles split their words");
    e->lanes_words = n_words;
    return BWG_OK;
}

extern "C" int bwg_ensemble_prepare(bwg_ens *e)
{
    TraceRange trace_("bwg_ensemble_prepare");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (e->lat || !e->want_jit_frank || e->jit_frank) return BWG_OK;
    return jit_frank_get(e->net, &e->jit_frank);
}

extern "C" int bwg_net_compile(bwg_net *n, uint32_t *built)
{
    TraceRange trace_("bwg_net_compile");
    if (!n) return fail(BWG_EINVAL, "null network");
    if (built) *built = 0;
    if (n->lat) return BWG_OK;
    const WmVariant *var = nullptr;
    const GenVariant *gv = nullptr;
    int rc = check_engine(n, BWG_ENGINE_BITWISE, &var, &gv);
    if (rc) return rc;
    bool gen = false, frank = false;
    jit_plan(n, BWG_ENGINE_BITWISE, var, false, true, &gen, &frank);
    rc = jit_build_codes(n, gen, frank);
    if (rc) return rc;
    if (built) *built = (gen ? BWG_JIT_GENERAL : 0u) | (frank ? BWG_JIT_FRANK : 0u);
    return BWG_OK;
}

extern "C" int bwg_ensemble_set_engine(bwg_ens *e, int32_t engine)
{
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (e->lat) return fail(BWG_EINVAL, "lattices have one engine");
    if (e->engine == BWG_ENGINE_PLAIN || (engine != BWG_ENGINE_BITWISE && engine != BWG_ENGINE_LANES))
        return fail(BWG_EINVAL, "only the bit-sliced and lanes engines share a state layout");
    if (engine == BWG_ENGINE_LANES && (e->gvar || e->jit))
        return fail(BWG_EINVAL, "the lanes engine runs Frank-family networks on their own kernel");
    if (engine == BWG_ENGINE_LANES) {
        const WmVariant *v = nullptr;
        const int rc = check_engine(e->net, BWG_ENGINE_LANES, &v);
        if (rc) return rc;
    }
    if (engine == BWG_ENGINE_BITWISE && !e->var && !e->gvar && !e->jit && !e->want_jit_frank) {
        e->var = pick_variant(e->net);
        if (!e->var) return fail(BWG_EUNSUPPORTED, "no bit-sliced kernel for this network");
    }
    e->engine = engine;
    return BWG_OK;
}

static int take_event(bwg_ens *e, hipEvent_t *ev)
{
    if (!e->spare.empty()) {
        *ev = e->spare.back();
        e->spare.pop_back();
        return BWG_OK;
    }
    HIP_TRY(hipEventCreate(ev));
    return BWG_OK;
}

int bwg::mark_begin(bwg_ens *e, hipStream_t s, hipEvent_t *ev)
{
    *ev = nullptr;
    if (!e->timed) return BWG_OK;
    int rc = take_event(e, ev);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(*ev, s));
    return BWG_OK;
}

int bwg::mark_end(bwg_ens *e, hipStream_t s, hipEvent_t ev)
{
    if (!e->timed) return BWG_OK;
    hipEvent_t stop;
    int rc = take_event(e, &stop);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(stop, s));
    e->marks.emplace_back(ev, stop);
    return BWG_OK;
}

extern "C" int bwg_ensemble_kernel_time(bwg_ens *e, double *ms, uint64_t *launches)
{
    if (!e || !ms || !launches) return fail(BWG_EINVAL, "null argument");
    if (!e->timed) return fail(BWG_EINVAL, "ensemble created without BWG_OPT_TIME_KERNELS");
    double total = 0;
    for (auto &m : e->marks) {
        HIP_TRY(hipEventSynchronize(m.second));
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, m.first, m.second));
        total += t;
        e->spare.push_back(m.first);
        e->spare.push_back(m.second);
    }
    *ms = total;
    *launches = e->marks.size();
    e->marks.clear();
    return BWG_OK;
}

extern "C" int bwg_ensemble_init(bwg_ens *e, int32_t mode, const int32_t *counts, void *stream)
{
    TraceRange trace_("bwg_ensemble_init");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    hipStream_t s = (hipStream_t)stream;
    const bwg_net *n = e->net;
    if (e->lat) return lat_init(e, mode, counts, s);
    int32_t c[BWG_MAX_SPECIES] = {};
    if (mode == BWG_INIT_FIXED) {
        if (!counts) return fail(BWG_EINVAL, "fixed init needs counts");
        int64_t sum = 0;
        for (int x = 0; x < n->S; ++x) {
            if (counts[x] < 0) return fail(BWG_EINVAL, "negative initial count");
            if (n->open && counts[x] > n->n_tot)
                return fail(BWG_ERANGE, "initial count %d above the cap n_tot = %lld", counts[x],
                            (long long)n->n_tot);
            c[x] = counts[x];
            sum += counts[x];
        }
        if (!n->open && sum != n->n_tot)
            return fail(BWG_EINVAL, "initial counts sum to %lld, not n_tot = %lld", (long long)sum,
                        (long long)n->n_tot);
    } else if (mode == BWG_INIT_MULTINOMIAL) {
        if (n->wide) return fail(BWG_EINVAL, "the multinomial start is for the Frank species");
    } else {
        return fail(BWG_EINVAL, "unknown init mode %d", mode);
    }
    if (e->engine != BWG_ENGINE_PLAIN) {
        if (mode == BWG_INIT_FIXED)
            HIP_TRY(launch_init_fixed(e->planes, n->S, e->nb, e->wp, e->M, c, e->E, e->Et, e->real,
                                      s));
        else
            HIP_TRY(launch_init_multinomial(e->planes, e->nb, e->wp, e->M, n->n_tot, e->seed,
                                            e->net_id, e->E, e->Et, e->real, s));
    } else {
        HIP_TRY(launch_plain_init(e->counts, 32 * e->wp, mode == BWG_INIT_FIXED ? 0 : 1, c,
                                  n->n_tot, e->seed, e->net_id, e->E, e->Et, e->real, s));
    }
    HIP_TRY(launch_fill_u64(e->adv_dev, 1, 0, s));
    e->t_now = 0;
    e->adv = 0;
    e->lag = 0;
    e->pending = 0;
    e->zE = 0;
    e->inited = true;
    return BWG_OK;
}

void bwg::note_scheduled(bwg_ens *e, uint64_t kmin, uint64_t kmax)
{
    e->pending = e->lag + kmax;
    e->lag += kmax - kmin;
}

void bwg::note_ran(bwg_ens *e, uint64_t max_events)
{
    if (max_events == 0 || max_events >= e->pending)
        e->pending = 0;
    else
        e->pending -= max_events;
}

// One launch of the pending events of every word, at most max_events each
// (0: all of them).
static int launch_events(bwg_ens *e, uint64_t max_events, hipStream_t s)
{
    const bwg_net *n = e->net;
    if (e->engine != BWG_ENGINE_PLAIN) {
        WmArgs a{};
        a.planes = e->planes;
        a.E = e->E;
        a.Etgt = e->Et;
        a.real = e->real;
        a.wp = e->wp;
        a.n_words = (e->M + 31) / 32;
        a.M = e->M;
        a.seed = e->seed;
        a.max_events = max_events;
        a.net_id = e->net_id;
        a.B = n->q.B;
        a.cu = n->shape.cu;
        a.fa = n->shape.fa;
        a.fi = n->shape.fi;
        a.nb_mem = e->nb;
        a.zs = e->zs;
        a.ztab = (const uint32_t *)e->table;
        a.zbase = e->zbase;
        a.zlen = e->zs ? e->zlen : 0;
        if (a.zs && !a.zlen) return fail(BWG_EINVAL, "shared thresholds not staged");
        const bool frank_jit = e->engine == BWG_ENGINE_BITWISE && e->want_jit_frank &&
                               e->block <= 0;
        if (frank_jit && !e->jit_frank) {
            const int jrc = jit_frank_get(e->net, &e->jit_frank);
            if (jrc) return jrc;
        }
        hipEvent_t ev = nullptr;
        int rc = mark_begin(e, s, &ev);
        if (rc) return rc;
        if (e->engine == BWG_ENGINE_LANES)
            HIP_TRY(launch_wm_lanes(a, s));
        else if (frank_jit)
            HIP_TRY(jit_launch(e->jit_frank, a, s));
        else if (e->jit)
            HIP_TRY(jit_launch(e->jit, a, s));
        else if (e->gvar)
            HIP_TRY(e->gvar->fn(a, n->gen, s));
        else if (e->var)
            HIP_TRY(e->var->fn(a, s, e->block, e->word_bits));
        else
            return fail(BWG_EUNSUPPORTED, "no kernel for this ensemble's engine and options");
        rc = mark_end(e, s, ev);
        if (rc) return rc;
    } else {
        PlainArgs a{};
        a.counts = e->counts;
        a.E = e->E;
        a.Etgt = e->Et;
        a.real = e->real;
        a.M = e->M;
        a.seed = e->seed;
        a.max_events = max_events;
        a.net_id = e->net_id;
        a.B = n->q.B;
        a.R = n->R;
        for (int j = 0; j < n->R; ++j) a.rx[j] = n->prx[j];
        hipEvent_t ev = nullptr;
        int rc = mark_begin(e, s, &ev);
        if (rc) return rc;
        HIP_TRY(launch_plain(a, s, e->block));
        rc = mark_end(e, s, ev);
        if (rc) return rc;
    }
    note_ran(e, max_events);
    return BWG_OK;
}

// Shared-threshold ensembles move in lockstep (every replica at event zE):
// run up to max_events (0: all) of the pending events in launches of at most
// the table's capacity, each preceded by the fill of its thresholds.
static int run_shared(bwg_ens *e, uint64_t max_events, hipStream_t s)
{
    uint64_t todo = e->pending;
    if (max_events && max_events < todo) todo = max_events;
    uint64_t cap = e->table_cap * 2;  // uint32 thresholds in the table region
    if (e->epl && e->epl < cap) cap = e->epl;
    while (todo) {
        const uint64_t len = todo < cap ? todo : cap;
        HIP_TRY(launch_shared_fill((uint32_t *)e->table, e->zE, len, e->seed, e->net_id, e->zs,
                                   s));
        e->zbase = e->zE;
        e->zlen = len;
        const int rc = launch_events(e, len, s);
        if (rc) return rc;
        e->zE += len;
        todo -= len;
    }
    return BWG_OK;
}

// Enqueue the event launches of a scheduled advance or step: enough launches
// of events_per_launch (if set) to cover the pending bound.
static int run_events(bwg_ens *e, hipStream_t s)
{
    if (e->zs) return run_shared(e, 0, s);
    if (!e->epl) return launch_events(e, 0, s);
    while (e->pending) {
        int rc = launch_events(e, e->epl, s);
        if (rc) return rc;
    }
    return BWG_OK;
}

// Philox4x32-10 on the host (Salmon et al., SC'11): the same rounds as the
// device function, for the one budget a shared-threshold advance draws.
static void host_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                        uint32_t out[4])
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// The budget every replica of a shared-threshold ensemble runs in an advance
// (the paper's one time step for all copies): one BUDGET draw at the
// reserved replica index 0xFFFFFFFF, inverted through the Poisson table.
static uint64_t shared_budget(const bwg_ens *e, const Table *t)
{
    uint32_t o[4];
    host_philox((uint32_t)e->adv, (DOM_BUDGET << 24) | ((uint32_t)(e->adv >> 32) & 0xFFFFu),
                0xFFFFFFFFu, e->net_id, e->seed, o);
    const uint64_t u = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    const uint64_t *T = t->vals.data();
    uint64_t lo = 0, hi = t->len;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (T[mid] <= u)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (uint64_t)(t->k_lo + (int64_t)lo);
}

int bwg::schedule_ensemble(bwg_ens *e, double t_end, hipStream_t s, uint64_t *kmin_out,
                           uint64_t *kmax_out)
{
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    if (!(t_end >= e->t_now)) return fail(BWG_EINVAL, "t_end %g before t_now %g", t_end, e->t_now);
    if (e->adv >= (1ull << 48)) return fail(BWG_ERANGE, "advance index overflow");
    if (e->zs) {
        // events arrive at rate Z / s, one budget for every replica; the
        // replicas stay in lockstep only if the last budget has run
        if (e->pending) return fail(BWG_EINVAL, "shared thresholds: run the pending events first");
        const double mu = ((double)e->zs / e->net->q.s) * (t_end - e->t_now);
        uint64_t K = 0;
        if (mu > 0) {
            const Table *t;
            const int rc = get_table(e->net, mu, &t, false);
            if (rc) return rc;
            K = shared_budget(e, t);
        }
        HIP_TRY(launch_budget(nullptr, 0, 0, K, 0, e->seed, e->net_id, e->adv_dev, e->M, e->E,
                              e->Et, s));
        HIP_TRY(launch_add_u64(e->adv_dev, 1, s));
        e->t_now = t_end;
        e->adv += 1;
        *kmin_out = *kmax_out = K;
        return BWG_OK;
    }
    const double mu = e->net->q.lambda * (t_end - e->t_now);
    uint64_t kmin = 0, kmax = 0;
    if (mu > 0) {
        const Table *t;
        int rc = get_table(e->net, mu, &t);
        if (rc) return rc;
        if (t->len > e->table_cap)
            return fail(BWG_ERANGE, "Poisson table of %llu entries exceeds capacity %llu",
                        (unsigned long long)t->len, (unsigned long long)e->table_cap);
        HIP_TRY(hipMemcpyAsync(e->table, t->host, t->len * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_budget(e->table, t->len, t->k_lo, 0, 1, e->seed, e->net_id, e->adv_dev,
                              e->M, e->E, e->Et, s));
        kmin = (uint64_t)t->k_lo;
        kmax = (uint64_t)t->k_lo + t->len;
    } else {
        HIP_TRY(launch_budget(nullptr, 0, 0, 0, 0, e->seed, e->net_id, e->adv_dev, e->M, e->E,
                              e->Et, s));
    }
    HIP_TRY(launch_add_u64(e->adv_dev, 1, s));
    e->t_now = t_end;
    e->adv += 1;
    *kmin_out = kmin;
    *kmax_out = kmax;
    return BWG_OK;
}

extern "C" int bwg_ensemble_schedule(bwg_ens *e, double t_end, void *stream)
{
    TraceRange trace_("bwg_ensemble_schedule");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (e->lat) return lat_schedule(e, t_end, (hipStream_t)stream);
    uint64_t kmin, kmax;
    int rc = schedule_ensemble(e, t_end, (hipStream_t)stream, &kmin, &kmax);
    if (rc) return rc;
    note_scheduled(e, kmin, kmax);
    return BWG_OK;
}

extern "C" int bwg_ensemble_run(bwg_ens *e, uint64_t max_events, void *stream)
{
    TraceRange trace_("bwg_ensemble_run");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    if (e->lat) return lat_run(e, max_events, (hipStream_t)stream);
    if (e->zs) return run_shared(e, max_events, (hipStream_t)stream);
    return launch_events(e, max_events, (hipStream_t)stream);
}

extern "C" int bwg_ensemble_pending(const bwg_ens *e, uint64_t *bound)
{
    if (!e || !bound) return fail(BWG_EINVAL, "null argument");
    *bound = e->pending;
    return BWG_OK;
}

extern "C" int bwg_ensemble_advance(bwg_ens *e, double t_end, void *stream)
{
    TraceRange trace_("bwg_ensemble_advance");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    hipStream_t s = (hipStream_t)stream;
    if (e->lat) {
        const int rc = lat_schedule(e, t_end, s);
        return rc ? rc : lat_run(e, 0, s);
    }
    uint64_t kmin, kmax;
    int rc = schedule_ensemble(e, t_end, s, &kmin, &kmax);
    if (rc) return rc;
    note_scheduled(e, kmin, kmax);
    return run_events(e, s);
}

extern "C" int bwg_ensemble_step(bwg_ens *e, uint64_t n_events, void *stream)
{
    TraceRange trace_("bwg_ensemble_step");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    hipStream_t s = (hipStream_t)stream;
    if (e->lat) {
        const int rc = lat_step_schedule(e, n_events, s);
        return rc ? rc : lat_run(e, 0, s);
    }
    if (e->zs && e->pending)
        return fail(BWG_EINVAL, "shared thresholds: run the pending events first");
    HIP_TRY(launch_budget(nullptr, 0, 0, n_events, 0, e->seed, e->net_id, e->adv_dev, e->M, e->E,
                          e->Et, s));
    note_scheduled(e, n_events, n_events);
    return run_events(e, s);
}

extern "C" int bwg_ensemble_read_counts(bwg_ens *e, int32_t *dst, void *stream)
{
    TraceRange trace_("bwg_ensemble_read_counts");
    if (!e || !dst) return fail(BWG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    if (e->lat) return lat_read_counts(e, dst, s);
    if (e->engine != BWG_ENGINE_PLAIN)
        HIP_TRY(launch_read_counts_planes(e->planes, e->net->S, e->nb, e->wp, e->M, dst, s));
    else
        HIP_TRY(launch_read_counts_plain(e->counts, e->M, dst, s));
    return BWG_OK;
}

extern "C" int bwg_ensemble_histogram(bwg_ens *e, int32_t n_bins, uint64_t *dst, void *stream)
{
    TraceRange trace_("bwg_ensemble_histogram");
    if (!e || !dst) return fail(BWG_EINVAL, "null argument");
    if (n_bins < 1 || n_bins > 16384) return fail(BWG_EINVAL, "n_bins %d out of range", n_bins);
    if (e->net->wide) return fail(BWG_EUNSUPPORTED, "the histogram is of the Frank species");
    hipStream_t s = (hipStream_t)stream;
    if (e->lat) return lat_histogram(e, n_bins, dst, s);
    HIP_TRY(launch_histogram(e->engine != BWG_ENGINE_PLAIN ? e->planes : nullptr, e->counts,
                             e->nb, e->wp, e->M, e->net->n_tot, n_bins, dst, s));
    return BWG_OK;
}

extern "C" int bwg_ensemble_record(bwg_ens *e, const double *t_grid, uint32_t n_points,
                                   const uint32_t *dev_sel, uint32_t n_sel, int32_t *dev_out,
                                   int32_t threshold, uint32_t *dev_first, void *stream)
{
    TraceRange trace_("bwg_ensemble_record");
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    if (e->lat) return fail(BWG_EUNSUPPORTED, "record runs on well-mixed ensembles");
    if (e->net->wide) return fail(BWG_EUNSUPPORTED, "record follows the Frank species");
    if (n_points && !t_grid) return fail(BWG_EINVAL, "null time grid");
    if (n_points && n_sel && (!dev_sel || !dev_out))
        return fail(BWG_EINVAL, "null selection or output");
    if (dev_first && threshold < 0) return fail(BWG_EINVAL, "negative threshold");
    if (n_points >= 0xFFFFFFFFu) return fail(BWG_EINVAL, "too many grid points");
    double t = e->t_now;
    for (uint32_t k = 0; k < n_points; ++k) {
        if (!(t_grid[k] >= t))
            return fail(BWG_EINVAL, "grid point %u (%g) before %g", k, t_grid[k], t);
        t = t_grid[k];
    }
    hipStream_t s = (hipStream_t)stream;
    const uint32_t *planes = e->engine != BWG_ENGINE_PLAIN ? e->planes : nullptr;
    for (uint32_t k = 0; k < n_points; ++k) {
        const int rc = bwg_ensemble_advance(e, t_grid[k], stream);
        if (rc) return rc;
        HIP_TRY(launch_gather_counts(planes, e->counts, e->nb, e->wp, e->M, dev_sel, n_sel,
                                     dev_out ? dev_out + (uint64_t)k * n_sel * 3 : nullptr, s));
        if (dev_first)
            HIP_TRY(launch_first_passage(planes, e->counts, e->nb, e->wp, e->M, threshold, k,
                                         dev_first, s));
    }
    return BWG_OK;
}

extern "C" int bwg_ensemble_read_events(bwg_ens *e, uint64_t *dev_events, uint64_t *dev_real,
                                        void *stream)
{
    if (!e) return fail(BWG_EINVAL, "null ensemble");
    hipStream_t s = (hipStream_t)stream;
    if (dev_events) HIP_TRY(launch_copy_u64(e->E, dev_events, e->M, s));
    if (dev_real) {
        if (e->engine != BWG_ENGINE_PLAIN)
            HIP_TRY(launch_copy_u64(e->real, dev_real, (e->M + 31) / 32, s));
        else
            HIP_TRY(launch_copy_u64(e->real, dev_real, e->M, s));
    }
    return BWG_OK;
}

extern "C" int bwg_ensemble_stats(bwg_ens *e, void *stream, bwg_stats *out)
{
    TraceRange trace_("bwg_ensemble_stats");
    if (!e || !out) return fail(BWG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_sum_u64(e->E, e->M, e->scratch, 0, s));
    HIP_TRY(launch_sum_u64(e->real, e->engine != BWG_ENGINE_PLAIN ? (e->M + 31) / 32 : e->M,
                           e->scratch, 1, s));
    uint64_t h[2];
    HIP_TRY(hipMemcpyAsync(h, e->scratch, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->n_replicas = e->M;
    out->advance_index = e->adv;
    out->t_now = e->t_now;
    out->events_total = h[0];
    out->real_total = h[1];
    return BWG_OK;
}
