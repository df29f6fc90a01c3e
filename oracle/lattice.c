/*
 * CPU oracle, compartment (lattice) version -- TEST INFRASTRUCTURE ONLY.
 *
 * The paper presents the bitwise method for a well-mixed reactor and names
 * non-well-mixed systems, ensembles of small compartments, as the
 * motivation (Sec. 1, Sec. 6).  The reading implemented here:
 *
 *   - Lx x Ly periodic sites; each site holds counts (L, D, A) with the site
 *     total capped at T = 2^P - 1 (P bit planes per species);
 *   - in every site the Frank reactions run with integer weights c_j h_j of
 *     the site counts (the well-mixed rule, Sec. 3, Eq. (7));
 *   - every molecule hops to each of its 4 neighbours at rate d (weight
 *     c_hop per molecule); a hop into a full site (total T) does nothing;
 *   - uniformisation by components: a reaction component per site of weight
 *     W_R = 2^B_R >= the largest site weight sum, and a hop component per
 *     (site, direction) of weight W_H = (T+1) c_hop; C = S (W_R + 4 W_H).
 *     Each event picks component k uniform in [0, C), shared by the replicas
 *     of one component group (2048 consecutive replicas), then within it
 *       reaction: threshold n uniform in [0, 2^B_R) per replica, first
 *                 crossing of the site's cumulative weights (else null);
 *       hop:      j uniform in [0, T+1) per replica: A if j < n_A, L if
 *                 j < n_A + n_L, D if j < n_site, else null.
 *     Each replica's chain is exactly the uniformised CTMC of its lattice.
 *
 * Draws (Philox4x32-10, counter (c0, domain<<24 | ..., c2, net_id)):
 *   COMPONENT (5): c0 = event low 32, c1 = 5<<24 | attempt<<16 | event
 *                  bits 32..47, c2 = group; u = out0 | out1<<32; Lemire:
 *                  m = u * C (128-bit), reject if low64(m) < 2^64 mod C.
 *   EVENT (1):     the well-mixed plane draws; a hop uses planes 0..P-1.
 *   INIT (3):      site counts of A uniform in {lo..hi}: c0 = site,
 *                  c1 = 3<<24 | 1<<23 | attempt, c2 = replica; outputs
 *                  0..3 in turn, 32-bit Lemire with rejection.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t lx, ly, P, B_r;
    int64_t c[5];      /* weights of A->L, A->D, A+L->2L, A+D->2D, L+D->2A */
    int64_t c_hop;     /* per molecule per direction                        */
    uint64_t C;        /* total component weight                            */
} orc_lat;

static void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                   uint32_t out[4])
{
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

#define ORC_LAT_GROUP_SHIFT 11   /* 2048 replicas share a component sequence */

/* Component of event e of a group: k uniform in [0, C). */
uint64_t orc_lat_component(uint64_t seed, uint32_t net_id, uint32_t group, uint64_t e, uint64_t C)
{
    const unsigned __int128 two64 = (unsigned __int128)1 << 64;
    const uint64_t thresh = (uint64_t)(two64 % C);
    unsigned __int128 m = 0;
    /* attempts 0..255; the last is taken as it is (reached with probability
       below (C / 2^64)^255) */
    for (uint32_t attempt = 0; attempt < 256; ++attempt) {
        uint32_t o[4];
        philox((uint32_t)e, (5u << 24) | (attempt << 16) | (uint32_t)((e >> 32) & 0xFFFFu),
               group, net_id, seed, o);
        uint64_t u = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        m = (unsigned __int128)u * C;
        if ((uint64_t)m >= thresh) break;
    }
    return (uint64_t)(m >> 64);
}

/* Uniform integer in [lo, hi] for (replica, site), exact. */
static int32_t init_count(uint64_t seed, uint32_t net_id, uint64_t i, uint32_t site, int32_t lo,
                          int32_t hi)
{
    const uint32_t R = (uint32_t)(hi - lo + 1);
    const uint32_t thresh = (uint32_t)(-R) % R;
    for (uint32_t attempt = 0; attempt < 65536; ++attempt) {
        uint32_t o[4];
        philox(site, (3u << 24) | (1u << 23) | attempt, (uint32_t)i, net_id, seed, o);
        for (int k = 0; k < 4; ++k) {
            uint64_t m = (uint64_t)o[k] * R;
            if ((uint32_t)m >= thresh) return lo + (int32_t)(m >> 32);
        }
    }
    return lo; /* 262144 rejections in a row: probability below 2^-1000000 */
}

/* Replicas first + k*stride, k < n: L = D = 0, A uniform in {lo..hi}. */
void orc_lat_init_uniform(uint64_t seed, uint32_t net_id, uint64_t first, uint64_t stride,
                          uint64_t n, int32_t S, int32_t lo, int32_t hi,
                          int32_t *sites /* [n][S][3] */)
{
    for (uint64_t k = 0; k < n; ++k)
        for (int32_t s = 0; s < S; ++s) {
            int32_t *c = sites + ((uint64_t)k * S + s) * 3;
            c[0] = 0;
            c[1] = 0;
            c[2] = init_count(seed, net_id, first + k * stride, (uint32_t)s, lo, hi);
        }
}

/* Bits 0..nb-1 of replica i's thresholds at event e (EVENT domain planes). */
static uint32_t plane_bits(uint64_t seed, uint32_t net_id, uint64_t i, uint64_t e, int nb)
{
    uint32_t G = (uint32_t)(i >> 5), lane = (uint32_t)(i & 31u), n = 0, o[4];
    for (int quad = 0; 4 * quad < nb; ++quad) {
        philox((uint32_t)e, (1u << 24) | ((uint32_t)quad << 16) | (uint32_t)((e >> 32) & 0xFFFFu),
               G, net_id, seed, o);
        for (int j = 0; j < 4 && 4 * quad + j < nb; ++j)
            n |= ((o[j] >> lane) & 1u) << (4 * quad + j);
    }
    return n;
}

/* Weights of the site reactions from the definition (Eq. (7) forms). */
static void site_weights(const orc_lat *L, const int32_t *c, int64_t w[5])
{
    const int64_t nl = c[0], nd = c[1], na = c[2];
    w[0] = L->c[0] * na;
    w[1] = L->c[1] * na;
    w[2] = L->c[2] * na * nl;
    w[3] = L->c[3] * na * nd;
    w[4] = L->c[4] * nl * nd;
}

static int32_t neighbour(const orc_lat *L, int32_t s, int dir)
{
    int32_t x = s % L->lx, y = s / L->lx;
    switch (dir) {
        case 0: x = (x + 1) % L->lx; break;
        case 1: x = (x + L->lx - 1) % L->lx; break;
        case 2: y = (y + 1) % L->ly; break;
        default: y = (y + L->ly - 1) % L->ly; break;
    }
    return y * L->lx + x;
}

/*
 * Run replicas first + k*stride, k < n: replica k runs events E0[k] ..
 * E0[k]+K[k]-1 on its sites[k][S][3].  real[k] counts state-changing events,
 * blocked[k] hops into full sites.  Returns 0, or -2 on a violated invariant.
 */
int orc_lat_run(const orc_lat *L, uint64_t seed, uint32_t net_id, uint64_t first,
                uint64_t stride, uint64_t n, int32_t *sites, const uint64_t *E0,
                const uint64_t *K, uint64_t *real, uint64_t *blocked, int n_threads)
{
    const int32_t S = L->lx * L->ly, T = (1 << L->P) - 1;
    const uint64_t WR = (uint64_t)1 << L->B_r, WH = (uint64_t)(T + 1) * (uint64_t)L->c_hop;
    const uint64_t Wsite = WR + 4 * WH;
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        int32_t *st = sites + (uint64_t)k * S * 3;
        const uint64_t i = first + (uint64_t)k * stride;
        uint64_t nreal = 0, nblk = 0;
        for (uint64_t t = 0; t < K[k]; ++t) {
            const uint64_t e = E0[k] + t;
            const uint64_t comp =
                orc_lat_component(seed, net_id, (uint32_t)(i >> ORC_LAT_GROUP_SHIFT), e, L->C);
            const int32_t s = (int32_t)(comp / Wsite);
            const uint64_t r = comp % Wsite;
            int32_t *c = st + 3 * s;
            if (r < WR) {
                const uint32_t thr = plane_bits(seed, net_id, i, e, L->B_r);
                int64_t w[5], m = 0;
                int rx = -1;
                site_weights(L, c, w);
                for (int j = 0; j < 5; ++j) {
                    m += w[j];
                    if ((int64_t)thr < m) { rx = j; break; }
                }
                if (rx == 0 || rx == 2) { c[0] += 1; c[2] -= 1; }
                else if (rx == 1 || rx == 3) { c[1] += 1; c[2] -= 1; }
                else if (rx == 4) { c[0] -= 1; c[1] -= 1; c[2] += 2; }
                if (rx >= 0) ++nreal;
            } else {
                const int dir = (int)((r - WR) / WH);
                const int32_t s2 = neighbour(L, s, dir);
                int32_t *c2 = st + 3 * s2;
                const uint32_t j = plane_bits(seed, net_id, i, e, L->P);
                int x = -1;
                if ((int32_t)j < c[2]) x = 2;
                else if ((int32_t)j < c[2] + c[0]) x = 0;
                else if ((int32_t)j < c[2] + c[0] + c[1]) x = 1;
                if (x >= 0) {
                    if (c2[0] + c2[1] + c2[2] >= T) {
                        ++nblk;
                    } else if (s2 == s) {
                        /* one site wide along this axis: the hop returns home */
                    } else {
                        c[x] -= 1;
                        c2[x] += 1;
                        ++nreal;
                    }
                }
            }
            if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] + c[1] + c[2] > T) { bad = 1; break; }
        }
        if (real) real[k] = nreal;
        if (blocked) blocked[k] = nblk;
    }
    return bad ? -2 : 0;
}
