/*
 * The paper's gain experiment on the host CPU (Sec. 5, "Efficiency gain"):
 * its network with the ghost reactions (Eqs. (1)-(6), integer weights 1,
 * total propensity Z = N(N-1)/2), M copies, T iterations, one random number
 * shared by all copies at every iteration (Sec. 4 step (a)), the copies
 * held in 64-bit words as in the paper.  Two engines on the same draws:
 *
 *   bwg_cpu_gain_bitwise -- the bit-parallel method: the counts of 64 copies
 *     bit-sliced in uint64 planes; per iteration the shared threshold n is
 *     compared with the cumulative weights A L, A L + A D, A L + A D + L D by
 *     successive borrow chains (the comparator/changer of Sec. 4), the
 *     counts change by masked ripple-carry additions (Sec. 4.1.1) and the
 *     pair counts by the incremental updates of App. B (a pair count takes
 *     the change of one species times the other's count), never a product of
 *     two counts after the first iteration;
 *   bwg_cpu_gain_serial -- the standard direct method run once per copy
 *     (Sec. 3): integer counts, the propensities from their definition, the
 *     CDF search, the update; every copy draws the iteration's number itself,
 *     as M separate runs do.
 *
 * Both give the same counts for every copy (the threshold of iteration e is
 * uniform on [0, Z) by 32-bit multiply-shift with rejection on output 0 of
 * the Philox4x32-10 call (e, 6 << 24 | attempt << 16 | e >> 32, 0, net_id)
 * keyed by the seed; the 256th attempt is taken as it is).  Used by the
 * benchmark only: the library's engines run on the GPU.
 */
#include <stdint.h>
#include <string.h>

#define MAXB 16   /* count planes */
#define MAXW 32   /* pair-count planes */

/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
 * multiplies by the Philox constants, the high halves xor-ed with the other
 * counter words and the round key; the key advances by the Weyl constants. */
static void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                   uint32_t out[4])
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t shared_n(uint64_t seed, uint32_t net_id, uint64_t e, uint32_t Z)
{
    const uint32_t thresh = (uint32_t)(0u - Z) % Z;
    uint64_t m = 0;
    uint32_t o[4];
    for (uint32_t att = 0; att < 256; ++att) {
        philox((uint32_t)e, (6u << 24) | (att << 16) | (uint32_t)((e >> 32) & 0xFFFFu), 0u,
               net_id, seed, o);
        m = (uint64_t)o[0] * Z;
        if ((uint32_t)m >= thresh) break;
    }
    return (uint32_t)(m >> 32);
}

/* ---- bit-sliced helpers on uint64 planes (64 copies per word) ---------- */

/* x += d, d = +1 on p1, -1 on m1, +2 on p2 (disjoint masks), nb planes */
static inline __attribute__((always_inline)) void add_delta(uint64_t *x, int nb, uint64_t p1, uint64_t m1, uint64_t p2)
{
    uint64_t c = 0;
    for (int q = 0; q < nb; ++q) {
        const uint64_t v = q == 0 ? (p1 | m1) : (q == 1 ? (p2 | m1) : m1);
        const uint64_t s = x[q] ^ v ^ c;
        c = (x[q] & v) | (x[q] & c) | (v & c);
        x[q] = s;
    }
}

/* acc (w planes) += d * y, d = +1 on p1, -1 on m1, +2 on p2 (disjoint):
 * |d| y is y or y one plane up, negated as (magnitude ^ m1) + m1 */
static inline __attribute__((always_inline)) void add_scaled(uint64_t *acc, int w, const uint64_t *y, int nb, uint64_t p1, uint64_t m1,
                       uint64_t p2)
{
    const uint64_t one = p1 | m1;
    uint64_t c = m1;
    for (int q = 0; q < w; ++q) {
        const uint64_t lo = q < nb ? (y[q] & one) : 0;
        const uint64_t hi = (q >= 1 && q - 1 < nb) ? (y[q - 1] & p2) : 0;
        const uint64_t v = (lo | hi) ^ m1;
        const uint64_t s = acc[q] ^ v ^ c;
        c = (acc[q] & v) | (acc[q] & c) | (v & c);
        acc[q] = s;
    }
}

/* out (w planes) = x * y (schoolbook over nb-plane operands) */
static inline __attribute__((always_inline)) void mul(uint64_t *out, int w, const uint64_t *x, const uint64_t *y, int nb)
{
    memset(out, 0, sizeof(uint64_t) * w);
    for (int j = 0; j < nb; ++j) {
        uint64_t c = 0;
        for (int q = j; q < w; ++q) {
            const uint64_t v = (q - j < nb) ? (x[q - j] & y[j]) : 0;
            const uint64_t s = out[q] ^ v ^ c;
            c = (out[q] & v) | (out[q] & c) | (v & c);
            out[q] = s;
        }
    }
}

/* d -= p (w planes of p, bc planes of d); returns the borrow out */
static inline __attribute__((always_inline)) uint64_t sub_keep(uint64_t *d, int bc, const uint64_t *p, int w)
{
    uint64_t br = 0;
    for (int q = 0; q < bc; ++q) {
        const uint64_t v = q < w ? p[q] : 0;
        const uint64_t nb = (~d[q] & (v | br)) | (v & br);
        d[q] ^= v ^ br;
        br = nb;
    }
    return br;
}

static int bits(int64_t v)
{
    int b = 0;
    while (v >> b) ++b;
    return b ? b : 1;
}

/* One word of up to 64 copies (lanes), T iterations; nb count planes, the
 * pair counts and the comparisons over 2 nb planes (Z < 2^(2 nb - 1)).
 * Always inlined with a constant nb, so every plane loop has a fixed trip
 * count, as the paper's fixed-width words do. */
static inline __attribute__((always_inline)) void run_word(const int nb, uint64_t lanes,
                                                           uint64_t seed, uint32_t net_id,
                                                           uint32_t Z, const int32_t *init,
                                                           uint64_t T, int32_t *out)
{
    const int w = 2 * nb, bc = 2 * nb;
    uint64_t N[3][MAXB], P[3][MAXW];   /* P: A L, A D, L D */
    memset(N, 0, sizeof N);
    for (uint64_t l = 0; l < lanes; ++l)
        for (int x = 0; x < 3; ++x)
            for (int q = 0; q < nb; ++q) N[x][q] |= (uint64_t)((init[l * 3 + x] >> q) & 1) << l;
    mul(P[0], w, N[2], N[0], nb);
    mul(P[1], w, N[2], N[1], nb);
    mul(P[2], w, N[0], N[1], nb);
    for (uint64_t e = 0; e < T; ++e) {
        const uint32_t n = shared_n(seed, net_id, e, Z);
        uint64_t d[MAXW];
        for (int q = 0; q < bc; ++q) d[q] = ((n >> q) & 1u) ? ~0ull : 0ull;
        /* comparator / changer: first crossing of A L, + A D, + L D */
        const uint64_t lt1 = sub_keep(d, bc, P[0], w);
        const uint64_t lt2 = lt1 | sub_keep(d, bc, P[1], w);
        const uint64_t lt3 = lt2 | sub_keep(d, bc, P[2], w);
        const uint64_t m1 = lt1, m2 = lt2 & ~lt1, m3 = lt3 & ~lt2;
        /* App. B: species in order L, D, A; a pair count takes the change
         * of one species times the other's current count */
        add_scaled(P[0], w, N[2], nb, m1, m3, 0);      /* dL * A  (A not yet changed) */
        add_scaled(P[2], w, N[1], nb, m1, m3, 0);      /* dL * D  (D not yet changed) */
        add_delta(N[0], nb, m1, m3, 0);
        add_scaled(P[1], w, N[2], nb, m2, m3, 0);      /* dD * A */
        add_scaled(P[2], w, N[0], nb, m2, m3, 0);      /* dD * L' */
        add_delta(N[1], nb, m2, m3, 0);
        add_scaled(P[0], w, N[0], nb, 0, m1 | m2, m3); /* dA * L' */
        add_scaled(P[1], w, N[1], nb, 0, m1 | m2, m3); /* dA * D' */
        add_delta(N[2], nb, 0, m1 | m2, m3);
    }
    for (uint64_t l = 0; l < lanes; ++l)
        for (int x = 0; x < 3; ++x) {
            int32_t v = 0;
            for (int q = 0; q < nb; ++q) v |= (int32_t)((N[x][q] >> l) & 1u) << q;
            out[l * 3 + x] = v;
        }
}

/* Copies [0, M) from init[k*3 .. k*3+2] = (L, D, A), T iterations from
 * iteration index 0; final counts in out.  0, or -1 on bad sizes. */
int bwg_cpu_gain_bitwise(int64_t n_tot, uint64_t M, uint64_t seed, uint32_t net_id,
                         const int32_t *init, uint64_t T, int32_t *out)
{
    const int nb = bits(n_tot);
    const uint64_t Z64 = (uint64_t)n_tot * (uint64_t)(n_tot - 1) / 2;
    if (n_tot < 2 || nb > MAXB || 2 * nb > MAXW || Z64 >= (1ull << 32)) return -1;
    const uint32_t Z = (uint32_t)Z64;
    for (uint64_t g = 0; g < M; g += 64) {
        const uint64_t lanes = M - g < 64 ? M - g : 64;
        const int32_t *in = init + g * 3;
        int32_t *o = out + g * 3;
        switch (nb) {
#define BWG_NB_CASE(k) \
    case k: run_word(k, lanes, seed, net_id, Z, in, T, o); break;
            BWG_NB_CASE(2) BWG_NB_CASE(3) BWG_NB_CASE(4) BWG_NB_CASE(5) BWG_NB_CASE(6)
            BWG_NB_CASE(7) BWG_NB_CASE(8) BWG_NB_CASE(9) BWG_NB_CASE(10) BWG_NB_CASE(11)
            BWG_NB_CASE(12) BWG_NB_CASE(13) BWG_NB_CASE(14) BWG_NB_CASE(15) BWG_NB_CASE(16)
#undef BWG_NB_CASE
        default: return -1;
        }
    }
    return 0;
}

int bwg_cpu_gain_serial(int64_t n_tot, uint64_t M, uint64_t seed, uint32_t net_id,
                        const int32_t *init, uint64_t T, int32_t *out)
{
    const uint64_t Z64 = (uint64_t)n_tot * (uint64_t)(n_tot - 1) / 2;
    if (n_tot < 2 || Z64 >= (1ull << 32)) return -1;
    const uint32_t Z = (uint32_t)Z64;
    for (uint64_t k = 0; k < M; ++k) {
        int64_t L = init[k * 3], D = init[k * 3 + 1], A = init[k * 3 + 2];
        for (uint64_t e = 0; e < T; ++e) {
            const int64_t n = shared_n(seed, net_id, e, Z);
            const int64_t a1 = A * L, a2 = a1 + A * D, a3 = a2 + L * D;
            if (n < a1) { ++L; --A; }
            else if (n < a2) { ++D; --A; }
            else if (n < a3) { --L; --D; A += 2; }
        }
        out[k * 3] = (int32_t)L;
        out[k * 3 + 1] = (int32_t)D;
        out[k * 3 + 2] = (int32_t)A;
    }
    return 0;
}
