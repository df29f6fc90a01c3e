// Device helpers of the general bit-sliced kernels (the precompiled one and
// the per-network ones compiled at run time).
#pragma once

#include "wm_device.h"

namespace bwg {

// x += delta with delta = +1 on p1, -1 on m1, +2 on p2, -2 on m2 (disjoint
// masks): two's complement addend planes 0: p1|m1, 1: p2|m1|m2, >= 2: m1|m2.
template <int NB>
__device__ __forceinline__ void add_delta(uint32_t (&x)[NB], uint32_t p1, uint32_t m1,
                                          uint32_t p2, uint32_t m2)
{
    const uint32_t a0 = p1 | m1, a1 = p2 | m1 | m2, an = m1 | m2;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const uint32_t v = q == 0 ? a0 : (q == 1 ? a1 : an);
        const uint32_t s = BWG_OP3(x[q], v, c, L_XOR3);
        if (q + 1 < NB) c = BWG_OP3(x[q], v, c, L_MAJ);
        x[q] = s;
    }
}

// acc += delta * y with delta = +1 on p1, -1 on m1, +2 on p2, -2 on m2
// (disjoint masks), y a non-negative NB-plane count, acc WP planes modulo
// 2^WP: the magnitude |delta| y is y or y shifted one plane up, negated as
// (magnitude ^ neg) + neg on the negative lanes, sign-extended.
template <int NB, int WP>
__device__ __forceinline__ void add_scaled(uint32_t (&acc)[WP], const uint32_t (&y)[NB],
                                           uint32_t p1, uint32_t m1, uint32_t p2, uint32_t m2)
{
    const uint32_t one = p1 | m1, two = p2 | m2, neg = m1 | m2;
    uint32_t c = neg;
#pragma unroll
    for (int q = 0; q < WP; ++q) {
        const uint32_t lo = q < NB ? (y[q] & one) : 0u;
        const uint32_t hi = (q >= 1 && q - 1 < NB) ? y[q - 1] : 0u;
        const uint32_t v = BWG_OP3(hi, two, lo, L_ANDOR) ^ neg;
        const uint32_t s = BWG_OP3(acc[q], v, c, L_XOR3);
        if (q + 1 < WP) c = BWG_OP3(acc[q], v, c, L_MAJ);
        acc[q] = s;
    }
}

// acc += 1 on a1, 3 on a3 (disjoint masks).
template <int WP>
__device__ __forceinline__ void add_one_three(uint32_t (&acc)[WP], uint32_t a1, uint32_t a3)
{
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < WP; ++q) {
        const uint32_t v = q == 0 ? (a1 | a3) : (q == 1 ? a3 : 0u);
        const uint32_t s = BWG_OP3(acc[q], v, c, L_XOR3);
        if (q + 1 < WP) c = BWG_OP3(acc[q], v, c, L_MAJ);
        acc[q] = s;
    }
}

// Lanes whose count x is at least the constant K (K < 2^NB): the complement
// of the borrow of x - K, one instruction per plane.
template <int NB, uint32_t K>
__device__ __forceinline__ uint32_t geq_const(const uint32_t (&x)[NB])
{
    uint32_t br = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) br = ((K >> q) & 1u) ? (~x[q] | br) : (~x[q] & br);
    return ~br;
}

// Counts of S species of word w (planes at or above the stored count are
// zero), and back after a launch that ran the word's events up to hi.
template <int S, int NB>
__device__ __forceinline__ void load_species(const WmArgs &a, uint64_t w, uint32_t (&N)[S][NB])
{
    if constexpr (S == 3) {
        load_word<NB>(a, w, N[0], N[1], N[2]);
    } else {
        const int nbm = a.nb_mem;
#pragma unroll
        for (int x = 0; x < S; ++x)
#pragma unroll
            for (int q = 0; q < NB; ++q)
                N[x][q] = q < nbm ? a.planes[((uint64_t)x * nbm + q) * a.wp + w] : 0u;
    }
}

template <int S, int NB>
__device__ __forceinline__ void store_species(const WmArgs &a, uint64_t w, uint32_t live,
                                              uint64_t hi, const uint32_t (&N)[S][NB])
{
    if constexpr (S == 3) {
        store_word<NB>(a, w, live, hi, N[0], N[1], N[2]);
    } else {
        const int nbm = a.nb_mem;
#pragma unroll
        for (int x = 0; x < S; ++x)
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q < nbm) a.planes[((uint64_t)x * nbm + q) * a.wp + w] = N[x][q];
        uint64_t *Ew = a.E + 32 * w;
        const uint64_t *T = a.Etgt + 32 * w;
        for (int l = 0; l < 32; ++l) {
            if (!((live >> l) & 1u)) continue;
            const uint64_t x = Ew[l], y = T[l];
            Ew[l] = hi < x ? x : (hi > y ? y : hi);
        }
    }
}

// Word loops of the per-network kernels: the event itself is a functor
// ev(d, act, N, nreal) that takes the threshold planes d (consumed), the
// active lanes and the counts N[species][plane], and adds its real lanes to
// nreal; ev.init(N) runs once per launch before the first event (the functor
// may keep quantities it updates from event to event).  S species (3 unless
// given).  gen_word: one thread per word, as wm_word.
template <int NB, int BC, int S = 3, typename Event>
__device__ __forceinline__ void gen_word(const WmArgs &a, uint64_t w, Event ev)
{
    if (w >= a.n_words) return;
    const uint32_t live = live_lanes(a, w);
    const uint64_t *E = a.E + 32 * w;
    const uint64_t *T = a.Etgt + 32 * w;
    const WordWindow win = word_window(a, E, T, live);
    uint32_t N[S][NB];
    load_species<S, NB>(a, w, N);
    if (win.lo < win.hi) {
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const int nq = (a.B + 3) / 4;
        uint32_t lastm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) lastm[j] = (4 * (nq - 1) + j < a.B) ? ~0u : 0u;
        uint64_t nreal = 0;
        uint64_t nxt = 0;  // next event at which the active lanes change
        uint32_t actc = 0;
        ev.init(N);
        for (uint64_t e = win.lo; e < win.hi; ++e) {
            if (e >= nxt) actc = lane_mask_next(E, T, win.pend, e, win.blo, nxt);
            const uint32_t act = actc;
            uint32_t d[BC];
            philox_planes<BC>(d, e, (uint32_t)w, a.net_id, k0, k1, nq, lastm);
            ev(d, act, N, nreal);
        }
        a.real[w] += nreal;
    }
    store_species<S, NB>(a, w, live, win.hi, N);
}

// gen_word_pc: the producer/consumer form of wm_word_pc (four waves per 128
// words, Philox planes handed over through rings of 2 x PH events in LDS, a
// barrier per PH events, the workgroup's largest window as step count).
template <int NB, int BC, int PH, int S = 3, typename Event>
__device__ __forceinline__ void gen_word_pc(const WmArgs &a, uint4 (*ring)[BC / 4][64],
                                            uint64_t *wave_span, Event ev)
{
    const int lane = threadIdx.x & 63;
    const int grp = (threadIdx.x >> 6) & 1;
    const bool producer = threadIdx.x < 128;
    ring += grp * 2 * PH;
    const uint64_t w = (uint64_t)blockIdx.x * 128 + grp * 64 + lane;
    const bool valid = w < a.n_words;
    const uint32_t live = valid ? live_lanes(a, w) : 0u;
    const uint64_t *E = a.E + 32 * (valid ? w : 0);
    const uint64_t *T = a.Etgt + 32 * (valid ? w : 0);
    const WordWindow win = word_window(a, E, T, live);
    const uint64_t lo = win.lo, hi = win.hi;
    {
        const uint64_t m = wave_max_u64(hi - lo);
        if (lane == 0) wave_span[threadIdx.x >> 6] = m;
    }
    __syncthreads();
    uint64_t span = wave_span[0];
    for (int i = 1; i < 4; ++i) span = wave_span[i] > span ? wave_span[i] : span;
    const uint64_t nsteps = (span + PH - 1) / PH;
    const int nq = (a.B + 3) / 4;

    if (producer) {
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        uint32_t lastm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) lastm[j] = (4 * (nq - 1) + j < a.B) ? ~0u : 0u;
        // quads past the network's threshold planes stay zero in every slot
        // (visible to the consumer after the first barrier)
        for (int h = 0; h < 2 * PH; ++h)
            for (int q4 = nq; q4 < BC / 4; ++q4) ring[h][q4][lane] = make_uint4(0, 0, 0, 0);
        for (uint64_t s = 0; s <= nsteps; ++s) {
            if (s < nsteps) {
                const int half = (int)(s & 1) * PH;
                for (int j = 0; j < PH; ++j) {
                    const uint64_t e = lo + s * PH + j;
                    if (e < hi) {
                        uint32_t n[BC];
                        philox_planes<BC>(n, e, (uint32_t)w, a.net_id, k0, k1, nq, lastm);
#pragma unroll
                        for (int q4 = 0; q4 < BC / 4; ++q4)
                            if (q4 < nq)
                                ring[half + j][q4][lane] =
                                    make_uint4(n[4 * q4], n[4 * q4 + 1], n[4 * q4 + 2], n[4 * q4 + 3]);
                    }
                }
            }
            __syncthreads();
        }
        return;
    }

    uint32_t N[S][NB];
    if (valid) {
        load_species<S, NB>(a, w, N);
    } else {
#pragma unroll
        for (int x = 0; x < S; ++x)
#pragma unroll
            for (int q = 0; q < NB; ++q) N[x][q] = 0u;
    }
    ev.init(N);
    uint64_t nreal = 0;
    uint64_t nxt = 0;  // next event at which the active lanes change
    uint32_t actc = 0;
    for (uint64_t s = 0; s <= nsteps; ++s) {
        if (s >= 1) {
            const int half = (int)((s - 1) & 1) * PH;
            for (int j = 0; j < PH; ++j) {
                const uint64_t e = lo + (s - 1) * PH + j;
                if (e < hi) {
                    if (e >= nxt) actc = lane_mask_next(E, T, win.pend, e, win.blo, nxt);
                    const uint32_t act = actc;
                    uint32_t d[BC];
#pragma unroll
                    for (int q4 = 0; q4 < BC / 4; ++q4) {
                        const uint4 v = ring[half + j][q4][lane];
                        d[4 * q4 + 0] = v.x;
                        d[4 * q4 + 1] = v.y;
                        d[4 * q4 + 2] = v.z;
                        d[4 * q4 + 3] = v.w;
                    }
                    ev(d, act, N, nreal);
                }
            }
        }
        __syncthreads();
    }
    if (valid) {
        if (lo < hi) a.real[w] += nreal;
        store_species<S, NB>(a, w, live, hi, N);
    }
}

}  // namespace bwg
