// The bit-sliced event loop of one word, shared by the per-ensemble kernels
// and the batched persistent kernel.  See wm_kernel.hip for what one event
// computes.
#pragma once

#include "bitops.h"
#include "bwg_internal.h"

namespace bwg {

// ---- subtraction of a shifted operand ------------------------------------
// d -= p << SH over planes [SH, BC); returns the final borrow.  Planes below
// SH are untouched (the operand is zero there).
template <int SH, int BC, int WP, bool KEEP>
__device__ __forceinline__ uint32_t sub_shifted(uint32_t (&d)[BC], const uint32_t (&p)[WP])
{
    uint32_t br = 0;
#pragma unroll
    for (int q = SH; q < BC; ++q) {
        const uint32_t v = (q - SH < WP) ? p[q - SH] : 0u;
        const uint32_t nb = BWG_OP3(d[q], v, br, L_BORROW);
        if (KEEP) d[q] = BWG_OP3(d[q], v, br, L_XOR3);
        br = nb;
    }
    return br;
}

// Run-time shift: dispatch to the compile-time subtraction.
template <int BC, int WP, bool KEEP, int SH = 0>
__device__ __forceinline__ uint32_t sub_dispatch(int sh, uint32_t (&d)[BC],
                                                 const uint32_t (&p)[WP])
{
    if constexpr (SH >= BC) {
        return 0u;
    } else {
        if (sh == SH) return sub_shifted<SH, BC, WP, KEEP>(d, p);
        return sub_dispatch<BC, WP, KEEP, SH + 1>(sh, d, p);
    }
}

template <int FA, int BC, int WP, bool KEEP>
__device__ __forceinline__ uint32_t sub_w(int sh, uint32_t (&d)[BC], const uint32_t (&p)[WP])
{
    if constexpr (FA >= 0)
        return sub_shifted<FA, BC, WP, KEEP>(d, p);
    else
        return sub_dispatch<BC, WP, KEEP>(sh, d, p);
}

// Active lanes of a word at event e: E_l <= e < Etgt_l.
__device__ __forceinline__ uint32_t lane_mask(const uint64_t *E, const uint64_t *T,
                                              uint32_t live, uint64_t e)
{
    uint32_t m = 0;
    for (int l = 0; l < 32; ++l) {
        if (!((live >> l) & 1u)) continue;
        const uint64_t a = E[l], b = T[l];
        m |= (a <= e && e < b) ? (1u << l) : 0u;
    }
    return m;
}

// One word (32 replicas) of an ensemble: run its pending events.
// NB count planes, BC = 4 * (quads of threshold planes), FA product shift
// (-1: run time), CU unimolecular weight (-1: run time).
template <int NB, int BC, int FA, int CU>
__device__ __forceinline__ void wm_word(const WmArgs &a, const uint64_t w)
{
    static_assert(BC % 4 == 0, "threshold planes come in Philox quads");
    constexpr int WP = 2 * NB - 2 > 1 ? 2 * NB - 2 : 2;   // product planes
    constexpr int WD = NB + 2;                             // product-delta planes
    if (w >= a.n_words) return;

    const uint64_t rem = a.M - 32 * w;
    const uint32_t live = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    const uint64_t *E = a.E + 32 * w;
    const uint64_t *T = a.Etgt + 32 * w;

    // event window of this word over its pending lanes (E_l < Etgt_l); a
    // lane that has finished its budget never limits the window
    uint64_t lo = ~0ull, hi = 0, blo = 0, bhi = ~0ull;
    uint32_t pend = 0;
    for (int l = 0; l < 32; ++l) {
        if (!((live >> l) & 1u)) continue;
        const uint64_t x = E[l], y = T[l];
        if (x >= y) continue;
        pend |= 1u << l;
        lo = x < lo ? x : lo;
        blo = x > blo ? x : blo;
        hi = y > hi ? y : hi;
        bhi = y < bhi ? y : bhi;
    }
    if (!pend) lo = hi = 0;
    if (a.max_events && hi > lo + a.max_events) hi = lo + a.max_events;

    // load occupancies (species order L, D, A); planes at or above the
    // stored count are zero
    uint32_t L[NB], D[NB], A[NB];
    const uint32_t *pl = a.planes;
    const int nbm = a.nb_mem;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const bool in = q < nbm;
        L[q] = in ? pl[((uint64_t)0 * nbm + q) * a.wp + w] : 0u;
        D[q] = in ? pl[((uint64_t)1 * nbm + q) * a.wp + w] : 0u;
        A[q] = in ? pl[((uint64_t)2 * nbm + q) * a.wp + w] : 0u;
    }

    if (lo < hi) {
        // pair counts and the unimolecular weight, recomputed once per launch
        uint32_t PAL[WP], PAD[WP], PLD[WP];
        mul_planes<NB, WP>(PAL, A, L);
        mul_planes<NB, WP>(PAD, A, D);
        mul_planes<NB, WP>(PLD, L, D);
        uint32_t U[BC];
#pragma unroll
        for (int q = 0; q < BC; ++q) U[q] = 0;
        const uint32_t cu = CU >= 0 ? (uint32_t)CU : a.cu;
#pragma unroll
        for (int k = 0; k < BC; ++k) {
            if ((cu >> k) & 1u) {
                uint32_t c = 0;
#pragma unroll
                for (int q = k; q < BC; ++q) {
                    const uint32_t v = (q - k < NB) ? A[q - k] : 0u;
                    const uint32_t s = BWG_OP3(U[q], v, c, L_XOR3);
                    c = BWG_OP3(U[q], v, c, L_MAJ);
                    U[q] = s;
                }
            }
        }
        // per-plane constants of U's update: -cu (minus the +1) and 2 cu
        const bool has_a = a.fa >= 0, has_i = a.fi >= 0;
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const uint32_t G = (uint32_t)w;
        // threshold planes in use: nq quads, the last one masked to plane B-1
        const int nq = (a.B + 3) / 4;
        uint32_t lastm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) lastm[j] = (4 * (nq - 1) + j < a.B) ? ~0u : 0u;
        uint64_t nreal = 0;

        for (uint64_t e = lo; e < hi; ++e) {
            const uint32_t act = (e >= blo && e < bhi) ? pend : lane_mask(E, T, pend, e);

            // (a) threshold planes: plane q is output q mod 4 of the Philox
            // call with plane-quad q / 4; planes at or above B are zero
            uint32_t n[BC];
            const uint32_t e_lo = (uint32_t)e, e_hi = (uint32_t)(e >> 32) & 0xFFFFu;
#pragma unroll
            for (int q4 = 0; q4 < BC / 4; ++q4) {
                uint32_t o0 = 0, o1 = 0, o2 = 0, o3 = 0;
                if (q4 < nq)
                    philox4x32_10(e_lo, (DOM_EVENT << 24) | ((uint32_t)q4 << 16) | e_hi, G,
                                  a.net_id, k0, k1, o0, o1, o2, o3);
                if (q4 == nq - 1) {
                    o0 &= lastm[0];
                    o1 &= lastm[1];
                    o2 &= lastm[2];
                    o3 &= lastm[3];
                }
                n[4 * q4 + 0] = o0;
                n[4 * q4 + 1] = o1;
                n[4 * q4 + 2] = o2;
                n[4 * q4 + 3] = o3;
            }

            // (b)-(d) cumulative weights and first crossing
            uint32_t br = 0;
#pragma unroll
            for (int q = 0; q < BC; ++q) br = BWG_OP3(n[q], U[q], br, L_BORROW);
            const uint32_t lt1 = br;  // n < U
            br = 0;                   // n -= 2U (in place)
#pragma unroll
            for (int q = 1; q < BC; ++q) {
                const uint32_t v = U[q - 1];
                const uint32_t nb = BWG_OP3(n[q], v, br, L_BORROW);
                n[q] = BWG_OP3(n[q], v, br, L_XOR3);
                br = nb;
            }
            const uint32_t lt2 = br;  // n < 2U
            uint32_t lt3 = lt2, lt4 = lt2, lt5;
            if (has_a) {
                lt3 = lt2 | sub_w<FA, BC, WP, true>(a.fa, n, PAL);
                lt4 = lt3 | sub_w<FA, BC, WP, true>(a.fa, n, PAD);
            }
            lt5 = lt4;
            if (has_i) lt5 = lt4 | sub_w<FA, BC, WP, false>(a.fi, n, PLD);

            const uint32_t mL = (lt1 | (lt3 & ~lt2)) & act;
            const uint32_t mD = ((lt2 & ~lt1) | (lt4 & ~lt3)) & act;
            const uint32_t mI = (lt5 & ~lt4) & act;
            const uint32_t mLD = mL | mD;
            nreal += (uint32_t)__builtin_popcount(mLD | mI);

            // (e) occupancies: keep the pre-event values for the products
            uint32_t L2[NB], D2[NB], A2[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                L2[q] = L[q];
                D2[q] = D[q];
                A2[q] = A[q];
            }
            add_pm1<NB>(L2, mL, mI);
            add_pm1<NB>(D2, mD, mI);
            add_m1_p2<NB>(A2, mLD, mI);

            // (f) products: P_AX += dA * X' + dX * A;  P_LD += dL * D' + dD * L
            {
                uint32_t t[WD];
                const uint32_t mLI = mL | mI, mDI = mD | mI;
                // P_AL
                {
                    uint32_t c = mLD;
#pragma unroll
                    for (int q = 0; q < WD; ++q) {
                        const uint32_t xq = q < NB ? L2[q] : 0u;
                        const uint32_t xm = (q >= 1 && q - 1 < NB) ? L2[q - 1] : 0u;
                        const uint32_t t1 = BWG_OP3(mI, xm, BWG_OP3(mLD, xq, 0u, L_ANDNOT), L_ANDOR);
                        const uint32_t t2 = q < NB ? BWG_OP3(A[q], mLI, mI, L_ANDXOR) : mI;
                        t[q] = BWG_OP3(t1, t2, c, L_XOR3);
                        c = BWG_OP3(t1, t2, c, L_MAJ);
                    }
                    add_sext<WP, WD>(PAL, t, mI);
                }
                // P_AD
                {
                    uint32_t c = mLD;
#pragma unroll
                    for (int q = 0; q < WD; ++q) {
                        const uint32_t xq = q < NB ? D2[q] : 0u;
                        const uint32_t xm = (q >= 1 && q - 1 < NB) ? D2[q - 1] : 0u;
                        const uint32_t t1 = BWG_OP3(mI, xm, BWG_OP3(mLD, xq, 0u, L_ANDNOT), L_ANDOR);
                        const uint32_t t2 = q < NB ? BWG_OP3(A[q], mDI, mI, L_ANDXOR) : mI;
                        t[q] = BWG_OP3(t1, t2, c, L_XOR3);
                        c = BWG_OP3(t1, t2, c, L_MAJ);
                    }
                    add_sext<WP, WD>(PAD, t, mI);
                }
                // P_LD
                {
                    uint32_t c = mI;
#pragma unroll
                    for (int q = 0; q < WD; ++q) {
                        const uint32_t t1 = q < NB ? BWG_OP3(D2[q], mLI, mI, L_ANDXOR) : mI;
                        const uint32_t t2 = q < NB ? BWG_OP3(L[q], mDI, mI, L_ANDXOR) : mI;
                        t[q] = BWG_OP3(t1, t2, c, L_XOR3);
                        c = BWG_OP3(t1, t2, c, L_MAJ);
                    }
                    add_sext<WP, WD>(PLD, t, mI);
                }
            }
            // U += cu * dA with dA = -1 on mLD, +2 on mI: addend planes are the
            // bits of -cu (two's complement, the +1 as carry-in) on mLD and of
            // 2 cu on mI
            if (cu) {
                uint32_t c = mLD;
#pragma unroll
                for (int q = 0; q < BC; ++q) {
                    uint32_t v;
                    if constexpr (CU >= 0) {
                        constexpr uint32_t ncu = ~(uint32_t)CU, dcu = 2u * (uint32_t)CU;
                        const bool bn = (ncu >> q) & 1u, bd = (dcu >> q) & 1u;
                        v = bn ? (bd ? (mLD | mI) : mLD) : (bd ? mI : 0u);
                    } else {
                        const uint32_t neg = ((cu >> q) & 1u) ? 0u : mLD;
                        const uint32_t dbl = (q >= 1 && ((cu >> (q - 1)) & 1u)) ? mI : 0u;
                        v = neg | dbl;
                    }
                    const uint32_t s = BWG_OP3(U[q], v, c, L_XOR3);
                    if (q + 1 < BC) c = BWG_OP3(U[q], v, c, L_MAJ);
                    U[q] = s;
                }
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                L[q] = L2[q];
                D[q] = D2[q];
                A[q] = A2[q];
            }
        }
        a.real[w] += nreal;
    }

    // store occupancies and the new per-replica event counts
    uint32_t *po = a.planes;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (q < nbm) {
            po[((uint64_t)0 * nbm + q) * a.wp + w] = L[q];
            po[((uint64_t)1 * nbm + q) * a.wp + w] = D[q];
            po[((uint64_t)2 * nbm + q) * a.wp + w] = A[q];
        }
    }
    uint64_t *Ew = a.E + 32 * w;
    for (int l = 0; l < 32; ++l) {
        if (!((live >> l) & 1u)) continue;
        const uint64_t x = Ew[l], y = T[l];
        Ew[l] = hi < x ? x : (hi > y ? y : hi);
    }
}

}  // namespace bwg
