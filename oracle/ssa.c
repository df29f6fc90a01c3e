/*
 * CPU oracle: per-replica Gillespie direct method with integer counts.
 * TEST INFRASTRUCTURE ONLY -- linked by the tests, the smoke check and the
 * benchmark's CPU baseline, never by the product library.
 *
 * Each replica is simulated on its own, one event at a time, exactly as the
 * serial update rule of Sec. 3 of the paper describes it:
 *   1. draw a uniform integer n (here on [0, W), W = 2^B, see below);
 *   2. evaluate every weight w_j(N) = c_j h_j(N) from its definition
 *      (Eq. (7) gives the paper's h_j);
 *   3. walk the reactions in table order accumulating m = sum_{p<=r} w_p and
 *      stop at the first r with n < m (the CDF search of Eqs. (10)-(11));
 *      if no reaction is reached the event is null -- the role of the ghost
 *      reactions (4)-(6), which pad the total to a state-independent
 *      constant (Eq. (9));
 *   4. apply N <- N + nu_r (Eqs. (13)-(14)); check N >= 0 and that the
 *      molecule count is conserved.
 * Time enters only through the number of events each replica runs (the
 * budgets computed by the caller, see poisson.py).
 *
 * Open networks (reactions that need not conserve the molecule count, the
 * general networks the paper leaves to future work, Sec. 6): every species
 * count is capped at cap = n_tot; a selected reaction whose firing would
 * leave some count above the cap does nothing (a null event), which is the
 * chain of the network on the truncated state space {0 <= N_x <= cap}.
 * Step 4 then checks N >= 0 and N <= cap instead of conservation.
 *
 * Random numbers follow the draw contract written independently in
 * philox.py (Philox4x32-10, Salmon et al. SC'11):
 *   key      = (seed low 32 bits, seed high 32 bits)
 *   counter  = (c0, (domain << 24) | (quad << 16) | hi16, c2, net_id)
 *   EVENT  (1): c0 = event low 32, hi16 = event bits 32..47, c2 = replica/32;
 *               bit (replica mod 32) of output (q mod 4) of quad q/4 is bit q
 *               of n (B planes, up to 62: n is 64-bit).
 *   BUDGET (2): c0 = advance index low 32, c2 = replica; u = out0 | out1<<32.
 *   INIT   (3): c0 = chunk, c2 = replica.
 *   PLAIN  (4): c0 = (event/4) low 32, hi16 = bits 32..47 of event/4,
 *               c2 = replica; n = out[event mod 4] mod 2^B (B <= 32; the
 *               runner refuses wider weights with -4).
 *   SHARED (6): the paper's variant in which one n serves every copy at an
 *               event (Sec. 4, the remark after the bitwise step; Sec. 6):
 *               c0 = event low 32, quad field = attempt, c2 = 0; n uniform
 *               on [0, Z) by 32-bit multiply-shift with rejection on out0
 *               (the 256th attempt is taken as it is).  Z is the constant
 *               total weight when the ghost reactions make it state
 *               independent (the paper's Z, Eq. (9)), else W.  An advance
 *               of this variant draws one BUDGET for every copy, at replica
 *               index 0xFFFFFFFF, with mean (Z / s) (t_end - t_now): the
 *               paper's single time step shared by the copies (Eq. (12)).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_S 8
#define ORC_MAX_R 16

typedef struct {
    int32_t n_species;
    int32_t n_reactions;
    int32_t reactants[ORC_MAX_R][ORC_MAX_S];
    int32_t products[ORC_MAX_R][ORC_MAX_S];
    int64_t c[ORC_MAX_R];
    int32_t B;
    uint32_t z_shared;   /* Z of the SHARED draw */
    int64_t n_tot;       /* conserved count; the per-species cap if open */
    int32_t open;        /* 1: the count is not conserved (capped at n_tot) */
    int32_t reserved;
} orc_net;

enum { ORC_DRAW_EVENT = 1, ORC_DRAW_PLAIN = 4, ORC_DRAW_SHARED = 6 };

/* ---- Philox4x32-10 ---------------------------------------------------- */
static void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                   uint64_t seed, uint32_t out[4])
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

void orc_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    philox(ctr[0], ctr[1], ctr[2], ctr[3], seed, out);
}

/* n for replica i at event e, bit-plane contract (EVENT domain); B up to
 * 62 planes (weights beyond 32 bits need more than 8 quads). */
static uint64_t draw_event(uint64_t seed, uint32_t net_id, uint64_t i,
                           uint64_t e, int B)
{
    uint32_t G = (uint32_t)(i >> 5), lane = (uint32_t)(i & 31u), out[4];
    uint64_t n = 0;
    for (int quad = 0; 4 * quad < B; ++quad) {
        philox((uint32_t)e,
               (1u << 24) | ((uint32_t)quad << 16) | (uint32_t)((e >> 32) & 0xFFFFu),
               G, net_id, seed, out);
        for (int j = 0; j < 4 && 4 * quad + j < B; ++j)
            n |= (uint64_t)((out[j] >> lane) & 1u) << (4 * quad + j);
    }
    return n;
}

/* n for replica i at event e, one-replica-per-thread contract (PLAIN; one
 * 32-bit output, so B <= 32). */
static uint32_t draw_plain(uint64_t seed, uint32_t net_id, uint64_t i,
                           uint64_t e, int B)
{
    uint32_t out[4];
    uint64_t blk = e >> 2;
    philox((uint32_t)blk, (4u << 24) | (uint32_t)((blk >> 32) & 0xFFFFu),
           (uint32_t)i, net_id, seed, out);
    uint32_t v = out[e & 3u];
    return B >= 32 ? v : (v & ((1u << B) - 1u));
}

/* n shared by every replica at event e: uniform on [0, Z). */
uint32_t orc_draw_shared(uint64_t seed, uint32_t net_id, uint64_t e, uint32_t Z)
{
    const uint32_t thresh = (uint32_t)(0u - Z) % Z;
    uint64_t m = 0;
    uint32_t out[4];
    for (uint32_t attempt = 0; attempt < 256; ++attempt) {
        philox((uint32_t)e, (6u << 24) | (attempt << 16) | (uint32_t)((e >> 32) & 0xFFFFu), 0u,
               net_id, seed, out);
        m = (uint64_t)out[0] * Z;
        if ((uint32_t)m >= thresh) break;
    }
    return (uint32_t)(m >> 32);
}

/* h_j(N): product over reactants of C(N_X, r_X), r_X in {0,1,2}. */
static int64_t comb(const orc_net *net, int j, const int64_t *N)
{
    int64_t v = 1;
    for (int x = 0; x < net->n_species; ++x) {
        int r = net->reactants[j][x];
        if (r == 1) v *= N[x];
        else if (r == 2) v *= N[x] * (N[x] - 1) / 2;
    }
    return v;
}

/* CDF search (Eqs. (10)-(11)): first reaction r, in table order, with
 * n < sum_{p<=r} w_p(N); -1 (null event) if n is at or above the total. */
static int select_reaction(const orc_net *net, const int64_t *N, uint64_t n)
{
    int64_t m = 0;  /* weights are non-negative: m >= 0 */
    for (int j = 0; j < net->n_reactions; ++j) {
        m += net->c[j] * comb(net, j, N);
        if (n < (uint64_t)m) return j;
    }
    return -1;
}

/* One event of the direct method.  Returns the reaction index, -1 for a
 * null event, -3 for a selected reaction blocked by the cap (open networks;
 * the state is unchanged); returns -2 on an invariant violation. */
static int one_event(const orc_net *net, int64_t *N, uint64_t n)
{
    int r = select_reaction(net, N, n);
    if (r < 0) return -1;
    if (net->open) {
        /* a firing that would pass the cap does nothing */
        for (int x = 0; x < net->n_species; ++x)
            if (N[x] + net->products[r][x] - net->reactants[r][x] > net->n_tot) return -3;
    }
    int64_t tot = 0;
    for (int x = 0; x < net->n_species; ++x) {
        N[x] += net->products[r][x] - net->reactants[r][x];
        if (N[x] < 0 || (net->open && N[x] > net->n_tot)) return -2;
        tot += N[x];
    }
    if (!net->open && tot != net->n_tot) return -2;
    return r;
}

/* Ghost reactions (Eqs. (4)-(6)) select a reaction without changing the
 * state; only state-changing events count as real. */
static int changes_state(const orc_net *net, int r)
{
    for (int x = 0; x < net->n_species; ++x)
        if (net->products[r][x] != net->reactants[r][x]) return 1;
    return 0;
}

int orc_select(const orc_net *net, const int32_t *counts, uint64_t n)
{
    int64_t N[ORC_MAX_S];
    for (int x = 0; x < net->n_species; ++x) N[x] = counts[x];
    return select_reaction(net, N, n);
}

/*
 * Run replicas [first, first+n): replica first+k starts from counts[k][:]
 * with E0[k] events already done and runs K[k] more (event indices
 * E0[k] .. E0[k]+K[k]-1).  counts is updated in place, real[k] receives the
 * number of non-null events.  If traj != NULL it receives the state after
 * every event, traj[(k*traj_len + t)*S + x] for t < min(K[k], traj_len).
 * Returns 0, or -2 if an invariant failed.
 */
int orc_wm_run(const orc_net *net, uint64_t seed, uint32_t net_id,
               int draw_mode, uint64_t first, uint64_t n, int32_t *counts,
               const uint64_t *E0, const uint64_t *K, uint64_t *real,
               int32_t *traj, uint64_t traj_len, int n_threads)
{
    const int S = net->n_species;
    int bad = 0;
    if (draw_mode == ORC_DRAW_PLAIN && net->B > 32) return -4;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 32) reduction(| : bad)
#endif
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        int64_t N[ORC_MAX_S];
        for (int x = 0; x < S; ++x) N[x] = counts[k * S + x];
        uint64_t i = first + (uint64_t)k, nreal = 0;
        for (uint64_t t = 0; t < K[k]; ++t) {
            uint64_t e = E0[k] + t;
            uint64_t thr = draw_mode == ORC_DRAW_PLAIN
                               ? draw_plain(seed, net_id, i, e, net->B)
                               : draw_mode == ORC_DRAW_SHARED
                                     ? orc_draw_shared(seed, net_id, e, net->z_shared)
                                     : draw_event(seed, net_id, i, e, net->B);
            int r = one_event(net, N, thr);
            if (r == -2) { bad = 1; break; }
            if (r >= 0 && changes_state(net, r)) ++nreal;
            if (traj && t < traj_len)
                for (int x = 0; x < S; ++x)
                    traj[((uint64_t)k * traj_len + t) * S + x] = (int32_t)N[x];
        }
        for (int x = 0; x < S; ++x) counts[k * S + x] = (int32_t)N[x];
        if (real) real[k] = nreal;
    }
    return bad ? -2 : 0;
}

/* Event budgets: K = k_lo + #{j : T[j] <= u}, u the BUDGET-domain uniform. */
void orc_budget(uint64_t seed, uint32_t net_id, uint64_t advance,
                uint64_t first, uint64_t n, const uint64_t *T, uint64_t L,
                int64_t k_lo, uint64_t *K_out)
{
    for (uint64_t k = 0; k < n; ++k) {
        uint32_t out[4];
        philox((uint32_t)advance,
               (2u << 24) | (uint32_t)((advance >> 32) & 0xFFFFu),
               (uint32_t)(first + k), net_id, seed, out);
        uint64_t u = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
        /* count entries <= u (T is non-decreasing) */
        uint64_t lo = 0, hi = L;
        while (lo < hi) {
            uint64_t mid = (lo + hi) / 2;
            if (T[mid] <= u) lo = mid + 1; else hi = mid;
        }
        K_out[k] = (uint64_t)(k_lo + (int64_t)lo);
    }
}

/* Multinomial initial state of the paper's experiment: each of n_tot
 * molecules is L, D or A with probabilities 1/4, 1/4, 1/2, from two random
 * bits (00 -> L, 01 -> D, 1x -> A); molecule m uses bits 2(m mod 64) and
 * 2(m mod 64)+1 of the 128-bit INIT draw with chunk m/64.  Species order of
 * counts is (L, D, A). */
void orc_init_multinomial(uint64_t seed, uint32_t net_id, uint64_t first,
                          uint64_t n, int64_t n_tot, int32_t *counts)
{
    for (uint64_t k = 0; k < n; ++k) {
        int32_t c[3] = {0, 0, 0};
        uint32_t out[4] = {0, 0, 0, 0};
        for (int64_t m = 0; m < n_tot; ++m) {
            if (m % 64 == 0)
                philox((uint32_t)(m / 64), 3u << 24, (uint32_t)(first + k),
                       net_id, seed, out);
            int bit = (int)(2 * (m % 64));
            uint32_t v = (out[bit / 32] >> (bit % 32)) & 3u;
            if (v == 0) c[0]++;
            else if (v == 1) c[1]++;
            else c[2]++;
        }
        counts[3 * k + 0] = c[0];
        counts[3 * k + 1] = c[1];
        counts[3 * k + 2] = c[2];
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
