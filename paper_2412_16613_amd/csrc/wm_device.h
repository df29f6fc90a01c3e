// The bit-sliced event loop of one word, shared by the per-ensemble kernels
// and the batched persistent kernel.  See wm_kernel.hip for what one event
// computes.
#pragma once

#include "bitops.h"
#include "bwg_internal.h"

namespace bwg {

// The threshold every replica compares at event e in the shared-threshold
// variant (the paper's single n per iteration, Sec. 4): uniform on [0, Z)
// from output 0 of SHARED draws by 32-bit multiply-shift, rejecting the low
// halves below 2^32 mod Z (thresh); the 256th attempt is kept as it is.
__device__ __forceinline__ uint32_t shared_threshold(uint64_t seed, uint32_t net_id, uint64_t e,
                                                     uint32_t Z, uint32_t thresh)
{
    uint64_t m = 0;
    for (uint32_t attempt = 0; attempt < 256; ++attempt) {
        uint32_t o0, o1, o2, o3;
        philox4x32_10((uint32_t)e, (DOM_SHARED << 24) | (attempt << 16) | ((uint32_t)(e >> 32) & 0xFFFFu),
                      0u, net_id, (uint32_t)seed, (uint32_t)(seed >> 32), o0, o1, o2, o3);
        m = (uint64_t)o0 * Z;
        if ((uint32_t)m >= thresh) break;
    }
    return (uint32_t)(m >> 32);
}

// Shared threshold of event e from the table the host fills before each
// launch: shared-threshold replicas move in lockstep, so every word's window
// is the table's [zbase, zbase + zlen).  The index is clamped to the table.
__device__ __forceinline__ uint32_t shared_at(const WmArgs &a, uint64_t e)
{
    const uint64_t k = e - a.zbase;
    return a.ztab[k < a.zlen ? k : a.zlen - 1];
}

// ---- subtraction of a shifted operand ------------------------------------
// d -= p << SH over planes [SH, NQ) (NQ <= BC, default all); returns the
// final borrow.  Planes below SH are untouched (the operand is zero there).
template <int SH, int BC, int WP, bool KEEP, int NQ = BC>
__device__ __forceinline__ uint32_t sub_shifted(uint32_t (&d)[BC], const uint32_t (&p)[WP])
{
    uint32_t br = 0;
#pragma unroll
    for (int q = SH; q < NQ; ++q) {
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

// Active lanes of a word at event e (E_l <= e < Etgt_l among pend) and, in
// nxt, the first event after e at which that set changes (~0: never), so
// that an event loop recomputes the set only there.  A word's 32 entries of
// E and Etgt are contiguous and 256-byte aligned (the arrays hold 32 entries
// for every word), so they are read with 16-byte loads, eight in flight;
// entries of lanes outside pend are read but ignored.  From blo on every
// pending lane has started and only the targets are needed.
__device__ __forceinline__ uint32_t lane_mask_next(const uint64_t *E, const uint64_t *T,
                                                   uint32_t pend, uint64_t e, uint64_t blo,
                                                   uint64_t &nxt)
{
    uint32_t m = 0;
    uint64_t nx = ~0ull;
    const uint4 *T4 = reinterpret_cast<const uint4 *>(T);
    if (e >= blo) {
#pragma unroll 1
        for (int g = 0; g < 2; ++g) {
            uint4 tv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) tv[j] = T4[8 * g + j];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int l = 16 * g + 2 * j + h;
                    const uint64_t y = h ? ((uint64_t)tv[j].w << 32 | tv[j].z)
                                         : ((uint64_t)tv[j].y << 32 | tv[j].x);
                    const bool on = ((pend >> l) & 1u) && e < y;
                    m |= on ? (1u << l) : 0u;
                    nx = (on && y < nx) ? y : nx;
                }
            }
        }
    } else {
        const uint4 *E4 = reinterpret_cast<const uint4 *>(E);
#pragma unroll 1
        for (int g = 0; g < 4; ++g) {
            uint4 ev[4], tv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ev[j] = E4[4 * g + j];
                tv[j] = T4[4 * g + j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int l = 8 * g + 2 * j + h;
                    const uint64_t x = h ? ((uint64_t)ev[j].w << 32 | ev[j].z)
                                         : ((uint64_t)ev[j].y << 32 | ev[j].x);
                    const uint64_t y = h ? ((uint64_t)tv[j].w << 32 | tv[j].z)
                                         : ((uint64_t)tv[j].y << 32 | tv[j].x);
                    const bool p = (pend >> l) & 1u;
                    m |= (p && x <= e && e < y) ? (1u << l) : 0u;
                    const uint64_t c = x > e ? x : (y > e ? y : ~0ull);
                    nx = (p && c < nx) ? c : nx;
                }
            }
        }
    }
    nxt = nx;
    return m;
}

// ---- pieces of one word's event loop ---------------------------------------

// Event window of a word over its pending lanes (E_l < Etgt_l): every
// pending event lies in [lo, hi) and every pending lane is active at the
// events of [blo, bhi); a lane that has finished its budget never limits it.
struct WordWindow {
    uint64_t lo, hi, blo, bhi;
    uint32_t pend;
};

__device__ __forceinline__ WordWindow word_window(const WmArgs &a, const uint64_t *E,
                                                  const uint64_t *T, uint32_t live)
{
    WordWindow v{~0ull, 0, 0, ~0ull, 0u};
    for (int l = 0; l < 32; ++l) {
        if (!((live >> l) & 1u)) continue;
        const uint64_t x = E[l], y = T[l];
        if (x >= y) continue;
        v.pend |= 1u << l;
        v.lo = x < v.lo ? x : v.lo;
        v.blo = x > v.blo ? x : v.blo;
        v.hi = y > v.hi ? y : v.hi;
        v.bhi = y < v.bhi ? y : v.bhi;
    }
    if (!v.pend) v.lo = v.hi = 0;
    if (a.max_events && v.hi > v.lo + a.max_events) v.hi = v.lo + a.max_events;
    return v;
}

// Occupancies of word w (species order L, D, A); planes at or above the
// stored count are zero.
template <int NB>
__device__ __forceinline__ void load_word(const WmArgs &a, uint64_t w, uint32_t (&L)[NB],
                                          uint32_t (&D)[NB], uint32_t (&A)[NB])
{
    const uint32_t *pl = a.planes;
    const int nbm = a.nb_mem;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const bool in = q < nbm;
        L[q] = in ? pl[((uint64_t)0 * nbm + q) * a.wp + w] : 0u;
        D[q] = in ? pl[((uint64_t)1 * nbm + q) * a.wp + w] : 0u;
        A[q] = in ? pl[((uint64_t)2 * nbm + q) * a.wp + w] : 0u;
    }
}

constexpr int bit_length(uint64_t v) { return v ? 1 + bit_length(v >> 1) : 0; }
// Planes of a two's complement number that holds every value of [lo, hi]
// (lo <= 0 <= hi), at least 2.
constexpr int signed_width(int64_t lo, int64_t hi)
{
    const uint64_t m = (uint64_t)(hi > -lo - 1 ? hi : -lo - 1);
    return bit_length(m) + 1 > 2 ? bit_length(m) + 1 : 2;
}

// Register widths of one word's event loop.  With the network's molecule
// count NT, product shifts FA, FI, unimolecular weight CU and selection
// planes BS all known at compile time (EXACT), every quantity is held in
// exactly the planes its largest value needs: U = CU N_A below CU NT, the
// pair counts below floor(NT/2) ceil(NT/2) (X + Y <= NT), and the second
// pair-count register holds Q_A = N_A (NT - N_A) = P_AL + P_AD, a function
// of N_A alone, so that S_4 = 2U + 2^FA Q_A is compared without S_3.
// Otherwise the widths follow the count planes NB and threshold planes BC.
template <int NB, int BC, int FA, int CU, int FI, int NT, int BS>
struct WmShape {
    static constexpr bool EXACT = NT > 0 && FA >= 0 && FI >= 0 && CU >= 0;  // and both
                                                                              // bimolecular
                                                                              // kinds present
    static constexpr int WP = EXACT ? (bit_length((uint64_t)(NT / 2) * (uint64_t)(NT - NT / 2)) > 1
                                           ? bit_length((uint64_t)(NT / 2) * (uint64_t)(NT - NT / 2))
                                           : 2)
                                    : (2 * NB - 2 > 1 ? 2 * NB - 2 : 2);
    static constexpr int UW = EXACT ? (bit_length((uint64_t)CU * (uint64_t)NT) > 0
                                           ? bit_length((uint64_t)CU * (uint64_t)NT)
                                           : 1)
                                    : BC;
    static constexpr int WD = NB + 2;  // product-delta planes
    // exact two's complement widths of the per-event changes (with their
    // carry-in convention) of P_AL: [-(NT - 1), 2NT - 4], of Q_A:
    // [-(2NT - 4), 2NT - 4] and of P_LD: [-NT, NT - 1]
    static constexpr int NTP = NT > 2 ? NT : 2;
    static constexpr int WD_AL = EXACT ? signed_width(-(int64_t)NTP + 1, 2 * (int64_t)NTP - 4) : WD;
    static constexpr int WD_QA = EXACT ? signed_width(-2 * (int64_t)NTP + 4, 2 * (int64_t)NTP - 4)
                                       : WD;
    static constexpr int WD_LD = EXACT ? signed_width(-(int64_t)NTP, (int64_t)NTP - 1) : WD;
    static constexpr int FMIN = FA < FI ? FA : FI;
    static_assert(!EXACT || (BS <= BC && UW < BS), "selection planes");
};

// Pair counts and the unimolecular weight U = cu N_A (UW planes), recomputed
// once per launch from the occupancies; with QA the second pair count is
// Q_A = N_A N_D + N_A N_L instead of N_A N_D.
template <int NB, int UW, int WP, bool QA = false>
__device__ __forceinline__ void init_weights(const uint32_t (&L)[NB], const uint32_t (&D)[NB],
                                             const uint32_t (&A)[NB], uint32_t cu,
                                             uint32_t (&PAL)[WP], uint32_t (&PAD)[WP],
                                             uint32_t (&PLD)[WP], uint32_t (&U)[UW])
{
    constexpr int BC = UW;
    mul_planes<NB, WP>(PAL, A, L);
    mul_planes<NB, WP>(PAD, A, D);
    if constexpr (QA) add_sext<WP, WP>(PAD, PAL, 0u);
    mul_planes<NB, WP>(PLD, L, D);
#pragma unroll
    for (int q = 0; q < BC; ++q) U[q] = 0;
#pragma unroll
    for (int k = 0; k < BC && k < 32; ++k) {  // cu has 32 bits; U may have more planes
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
}

// Threshold planes of event e for word G from Philox: plane q is output
// q mod 4 of the call with plane-quad q / 4; planes at or above B are zero
// (lastm masks the last of the nq quads in use).
template <int BC>
__device__ __forceinline__ void philox_planes(uint32_t (&n)[BC], uint64_t e, uint32_t G,
                                              uint32_t net_id, uint32_t k0, uint32_t k1, int nq,
                                              const uint32_t (&lastm)[4])
{
    const uint32_t e_lo = (uint32_t)e, e_hi = (uint32_t)(e >> 32) & 0xFFFFu;
#pragma unroll
    for (int q4 = 0; q4 < BC / 4; ++q4) {
        uint32_t o0 = 0, o1 = 0, o2 = 0, o3 = 0;
        if (q4 < nq)
            philox4x32_10(e_lo, (DOM_EVENT << 24) | ((uint32_t)q4 << 16) | e_hi, G, net_id, k0, k1,
                          o0, o1, o2, o3);
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
}


// Occupancies and per-replica event counts back to memory after a launch
// that ran the word's events up to hi.
template <int NB>
__device__ __forceinline__ void store_word(const WmArgs &a, uint64_t w, uint32_t live,
                                           uint64_t hi, const uint32_t (&L)[NB],
                                           const uint32_t (&D)[NB], const uint32_t (&A)[NB])
{
    uint32_t *po = a.planes;
    const int nbm = a.nb_mem;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (q < nbm) {
            po[((uint64_t)0 * nbm + q) * a.wp + w] = L[q];
            po[((uint64_t)1 * nbm + q) * a.wp + w] = D[q];
            po[((uint64_t)2 * nbm + q) * a.wp + w] = A[q];
        }
    }
    uint64_t *Ew = a.E + 32 * w;
    const uint64_t *T = a.Etgt + 32 * w;
    for (int l = 0; l < 32; ++l) {
        if (!((live >> l) & 1u)) continue;
        const uint64_t x = Ew[l], y = T[l];
        Ew[l] = hi < x ? x : (hi > y ? y : hi);
    }
}

__device__ __forceinline__ uint32_t live_lanes(const WmArgs &a, uint64_t w)
{
    const uint64_t rem = a.M - 32 * w;
    return rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
}

// One word (32 replicas) of an ensemble: run its pending events.
// NB count planes, BC = 4 * (quads of threshold planes), FA product shift
// of the A + L and A + D weights and FI that of the L + D weight (-1: run
// time), CU unimolecular weight (-1: run time); SH: one shared threshold per
// event (a.zs != 0) instead of per-replica draws.
template <int NB, int BC, int FA, int CU, bool SH = false, int FI = FA, int NT = 0, int BS = BC>
__device__ __forceinline__ void wm_word(const WmArgs &a, const uint64_t w)
{
    static_assert(BC % 4 == 0, "threshold planes come in Philox quads");
    using Sh = WmShape<NB, BC, FA, CU, FI, NT, BS>;
    constexpr bool EXACT = Sh::EXACT;
    constexpr int WP = Sh::WP, WD = Sh::WD, UW = Sh::UW, FMIN = Sh::FMIN;
    constexpr int WD_AL = Sh::WD_AL, WD_QA = Sh::WD_QA, WD_LD = Sh::WD_LD;
    if (w >= a.n_words) return;

    const uint32_t live = live_lanes(a, w);
    const uint64_t *E = a.E + 32 * w;
    const uint64_t *T = a.Etgt + 32 * w;
    const WordWindow win = word_window(a, E, T, live);
    const uint64_t lo = win.lo, hi = win.hi;

    uint32_t L[NB], D[NB], A[NB];
    load_word<NB>(a, w, L, D, A);

    if (lo < hi) {
        uint32_t PAL[WP], PAD[WP], PLD[WP], U[UW];
        const uint32_t cu = CU >= 0 ? (uint32_t)CU : a.cu;
        init_weights<NB, UW, WP, EXACT>(L, D, A, cu, PAL, PAD, PLD, U);
        // the exact-width variants serve networks with both reactions
        const bool has_a = EXACT || a.fa >= 0, has_i = EXACT || a.fi >= 0;
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const uint32_t G = (uint32_t)w;
        // threshold planes in use: nq quads, the last one masked to plane B-1
        const int nq = (a.B + 3) / 4;
        uint32_t lastm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) lastm[j] = (4 * (nq - 1) + j < a.B) ? ~0u : 0u;
        uint32_t nv_next = SH ? shared_at(a, lo) : 0u;
        uint64_t nreal = 0;
        uint64_t nxt = 0;  // next event at which the active lanes change
        uint32_t actc = 0;

        for (uint64_t e = lo; e < hi; ++e) {
            if (e >= nxt) actc = lane_mask_next(E, T, win.pend, e, win.blo, nxt);
            const uint32_t act = actc;
            // (a) threshold planes
            uint32_t n[BC];
            if constexpr (SH) {
                // one n for every replica: plane q is all ones where bit q is
                // set; the next event's n is loaded while this one runs
                const uint32_t nv = nv_next;
                if (e + 1 < hi) nv_next = shared_at(a, e + 1);
#pragma unroll
                for (int q = 0; q < BC; ++q)
                    n[q] = q < 32 ? (uint32_t)((int32_t)(nv << (31 - q)) >> 31) : 0u;
            } else {
                philox_planes<BC>(n, e, G, a.net_id, k0, k1, nq, lastm);
            }
#include "wm_event_body.inc"
        }
        a.real[w] += nreal;
    }
    store_word<NB>(a, w, live, hi, L, D, A);
}

// Word widths other than 32 replicas per thread (WW = 16 or 64); the
// results are those of wm_word, since every draw is keyed by the 32-lane
// word and the lane.  WW = 64: thread t runs the 32-replica words 2t and
// 2t + 1 -- two states, one event loop over the union of their windows, each
// word with its own threshold planes and active lanes, the two event bodies
// in one basic block.  WW = 16: thread t runs the lanes 16 (t mod 2) .. +15
// of word t / 2: it loads the whole word but only its half's lanes are
// active (the other half's planes pass through unchanged), and it stores
// the planes back as 16-bit halves and adds its real events atomically, so
// the two threads of a word never write the same bytes.  The instructions
// per event are those of a 32-replica word (a 16-bit bit-plane operation
// issues at the 32-bit rate).
template <int NB, int BC, int FA, int CU, bool SH, int FI, int NT, int BS, int WW>
__device__ __forceinline__ void wm_word_w(const WmArgs &a, const uint64_t t)
{
    static_assert(WW == 16 || WW == 64, "16 or 64 replicas per thread");
    static_assert(BC % 4 == 0, "threshold planes come in Philox quads");
    using Sh = WmShape<NB, BC, FA, CU, FI, NT, BS>;
    constexpr bool EXACT = Sh::EXACT;
    constexpr int WP = Sh::WP, WD = Sh::WD, UW = Sh::UW, FMIN = Sh::FMIN;
    constexpr int WD_AL = Sh::WD_AL, WD_QA = Sh::WD_QA, WD_LD = Sh::WD_LD;
    constexpr int WPT = WW == 64 ? 2 : 1;
    uint64_t wv[WPT];
    uint32_t livev[WPT];
    WordWindow win[WPT];
    uint64_t lo = ~0ull, hi = 0;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
        wv[i] = WW == 64 ? 2 * t + i : t >> 1;
        const bool valid = wv[i] < a.n_words;
        uint32_t lv = valid ? live_lanes(a, wv[i]) : 0u;
        if (WW == 16) lv &= (t & 1) ? 0xFFFF0000u : 0x0000FFFFu;
        livev[i] = lv;
        win[i] = word_window(a, a.E + 32 * (valid ? wv[i] : 0), a.Etgt + 32 * (valid ? wv[i] : 0),
                             lv);
        if (win[i].lo < win[i].hi) {
            lo = win[i].lo < lo ? win[i].lo : lo;
            hi = win[i].hi > hi ? win[i].hi : hi;
        }
    }
    if (hi == 0) lo = 0;
    if (wv[0] >= a.n_words) return;

    uint32_t Ls[WPT][NB], Ds[WPT][NB], As[WPT][NB];
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
        if (wv[i] < a.n_words) {
            load_word<NB>(a, wv[i], Ls[i], Ds[i], As[i]);
        } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) Ls[i][q] = Ds[i][q] = As[i][q] = 0u;
        }
    }
    uint64_t nrealv[WPT];
#pragma unroll
    for (int i = 0; i < WPT; ++i) nrealv[i] = 0;
    if (lo < hi) {
        uint32_t PALs[WPT][WP], PADs[WPT][WP], PLDs[WPT][WP], Us[WPT][UW];
        const uint32_t cu = CU >= 0 ? (uint32_t)CU : a.cu;
#pragma unroll
        for (int i = 0; i < WPT; ++i)
            init_weights<NB, UW, WP, EXACT>(Ls[i], Ds[i], As[i], cu, PALs[i], PADs[i], PLDs[i],
                                            Us[i]);
        const bool has_a = EXACT || a.fa >= 0, has_i = EXACT || a.fi >= 0;
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const int nq = (a.B + 3) / 4;
        uint32_t lastm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) lastm[j] = (4 * (nq - 1) + j < a.B) ? ~0u : 0u;
        uint32_t nv_next = SH ? shared_at(a, lo) : 0u;
        uint64_t nxt[WPT];
        uint32_t actc[WPT];
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
            nxt[i] = 0;
            actc[i] = 0;
        }
        for (uint64_t e = lo; e < hi; ++e) {
            uint32_t nsh[BC];
            if constexpr (SH) {
                const uint32_t nv = nv_next;
                if (e + 1 < hi) nv_next = shared_at(a, e + 1);
#pragma unroll
                for (int q = 0; q < BC; ++q)
                    nsh[q] = q < 32 ? (uint32_t)((int32_t)(nv << (31 - q)) >> 31) : 0u;
            }
#pragma unroll
            for (int i = 0; i < WPT; ++i) {
                const uint64_t *E = a.E + 32 * wv[i];
                const uint64_t *T = a.Etgt + 32 * wv[i];
                if (e >= nxt[i]) actc[i] = lane_mask_next(E, T, win[i].pend, e, win[i].blo, nxt[i]);
                const uint32_t act = actc[i];
                uint32_t n[BC];
                if constexpr (SH) {
#pragma unroll
                    for (int q = 0; q < BC; ++q) n[q] = nsh[q];
                } else {
                    philox_planes<BC>(n, e, (uint32_t)wv[i], a.net_id, k0, k1, nq, lastm);
                }
                uint32_t(&L)[NB] = Ls[i];
                uint32_t(&D)[NB] = Ds[i];
                uint32_t(&A)[NB] = As[i];
                uint32_t(&PAL)[WP] = PALs[i];
                uint32_t(&PAD)[WP] = PADs[i];
                uint32_t(&PLD)[WP] = PLDs[i];
                uint32_t(&U)[UW] = Us[i];
                uint64_t &nreal = nrealv[i];
#include "wm_event_body.inc"
            }
        }
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
        const uint64_t w = wv[i];
        if (w >= a.n_words) continue;
        if (WW == 16) {
            // this thread's half of every plane, and its lanes' event counts
            uint16_t *ph = reinterpret_cast<uint16_t *>(a.planes);
            const int nbm = a.nb_mem;
            const int sh = (t & 1) ? 16 : 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (q < nbm) {
                    ph[(((uint64_t)0 * nbm + q) * a.wp + w) * 2 + (t & 1)] = (uint16_t)(Ls[i][q] >> sh);
                    ph[(((uint64_t)1 * nbm + q) * a.wp + w) * 2 + (t & 1)] = (uint16_t)(Ds[i][q] >> sh);
                    ph[(((uint64_t)2 * nbm + q) * a.wp + w) * 2 + (t & 1)] = (uint16_t)(As[i][q] >> sh);
                }
            }
            uint64_t *Ew = a.E + 32 * w;
            const uint64_t *T = a.Etgt + 32 * w;
            for (int l = 0; l < 32; ++l) {
                if (!((livev[i] >> l) & 1u)) continue;
                const uint64_t x = Ew[l], y = T[l];
                Ew[l] = hi < x ? x : (hi > y ? y : hi);
            }
            if (nrealv[i]) atomicAdd((unsigned long long *)&a.real[w], (unsigned long long)nrealv[i]);
        } else {
            if (win[i].lo < win[i].hi) a.real[w] += nrealv[i];
            store_word<NB>(a, w, livev[i], hi, Ls[i], Ds[i], As[i]);
        }
    }
}

// 64-bit maximum over the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    for (int o = 32; o; o >>= 1) {
        const uint64_t u = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)v, o) |
                           ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o) << 32);
        v = u > v ? u : v;
    }
    return v;
}

// Producer/consumer form of wm_word for launches with fewer words than the
// chip has SIMDs.  A workgroup of four waves serves 128 words in two groups
// of 64: waves 0 and 1 draw the Philox threshold planes of their group's
// events into the group's ring in LDS, waves 2 and 3 run selection and
// updates on them, so a word's chain of events is split over two waves (and
// two SIMDs: the waves of a workgroup are spread over the CU's SIMDs).  A
// ring holds 2 halves of PH events; at step s the producer fills half s mod 2
// with events [s PH, (s+1) PH) of every word's window while the consumer runs
// the events of half (s-1) mod 2, and a barrier separates the steps.  The
// step count is the workgroup's largest window, so every wave meets every
// barrier.  Results are those of wm_word.
template <int NB, int BC, int FA, int CU, int PH, int FI = FA, int NT = 0, int BS = BC>
__device__ __forceinline__ void wm_word_pc(const WmArgs &a, uint4 (*ring)[BC / 4][64],
                                           uint64_t *wave_span)
{
    static_assert(BC % 4 == 0, "threshold planes come in Philox quads");
    using Sh = WmShape<NB, BC, FA, CU, FI, NT, BS>;
    constexpr bool EXACT = Sh::EXACT;
    constexpr int WP = Sh::WP, WD = Sh::WD, UW = Sh::UW, FMIN = Sh::FMIN;
    constexpr int WD_AL = Sh::WD_AL, WD_QA = Sh::WD_QA, WD_LD = Sh::WD_LD;
    const int lane = threadIdx.x & 63;
    const int grp = (threadIdx.x >> 6) & 1;
    const bool producer = threadIdx.x < 128;
    ring += grp * 2 * PH;
    const uint64_t w = (uint64_t)blockIdx.x * 128 + grp * 64 + lane;
    // words past the end take part in every barrier with an empty window
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
        const uint32_t G = (uint32_t)w;
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
                        philox_planes<BC>(n, e, G, a.net_id, k0, k1, nq, lastm);
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

    uint32_t L[NB], D[NB], A[NB];
    if (valid) {
        load_word<NB>(a, w, L, D, A);
    } else {
#pragma unroll
        for (int q = 0; q < NB; ++q) L[q] = D[q] = A[q] = 0u;
    }
    uint32_t PAL[WP], PAD[WP], PLD[WP], U[UW];
    const uint32_t cu = CU >= 0 ? (uint32_t)CU : a.cu;
    init_weights<NB, UW, WP, EXACT>(L, D, A, cu, PAL, PAD, PLD, U);
    // the exact-width variants serve networks with both reactions
    const bool has_a = EXACT || a.fa >= 0, has_i = EXACT || a.fi >= 0;
    uint64_t nreal = 0;
    uint64_t nxt = 0;  // next event at which the active lanes change
    uint32_t actc = 0;
    for (uint64_t s = 0; s <= nsteps; ++s) {
        if (s >= 1) {
            const int half = (int)((s - 1) & 1) * PH;
            // unrolled where the weights are compile-time: the PH events of
            // a step share registers without copies and the ring offsets are
            // constants (measured faster); the run-time weight variants,
            // whose shifted subtractions dispatch per shift, run slower
            // unrolled
            constexpr int UNR = (FA >= 0 && CU >= 0) ? PH : 1;
#pragma unroll UNR
            for (int j = 0; j < PH; ++j) {
                const uint64_t e = lo + (s - 1) * PH + j;
                if (e < hi) {
                    if (e >= nxt) actc = lane_mask_next(E, T, win.pend, e, win.blo, nxt);
                    const uint32_t act = actc;
                    uint32_t n[BC];
#pragma unroll
                    for (int q4 = 0; q4 < BC / 4; ++q4) {
                        const uint4 v = ring[half + j][q4][lane];
                        n[4 * q4 + 0] = v.x;
                        n[4 * q4 + 1] = v.y;
                        n[4 * q4 + 2] = v.z;
                        n[4 * q4 + 3] = v.w;
                    }
#include "wm_event_body.inc"
                }
            }
        }
        __syncthreads();
    }
    if (valid) {
        if (lo < hi) a.real[w] += nreal;
        store_word<NB>(a, w, live, hi, L, D, A);
    }
}

}  // namespace bwg

namespace bwg {

// One word of an ensemble with one replica per thread ("lanes" engine): the
// 32 threads of one half of a wave hold the word's 32 replicas as int32
// counts, unpacked from the bit planes at the start and packed back at the
// end.  Every event uses the same EVENT planes as wm_word, and each thread
// compares its own threshold with the cumulative weights in integer
// arithmetic, so the result is bit for bit the one wm_word gives.
//
// The planes are drawn for runs of 32 events: thread t makes the nq =
// ceil(B / 4) Philox calls of event e0 + t, transposes the 32 x 32 bit matrix
// of its event's planes in registers (plane q's bit l becomes bit q of row l:
// replica l's threshold) and stores the 32 thresholds in sq, this half's LDS
// (event g's row at [36 g, 36 g + 32); the stride of 36 words spreads the
// rows' stores over the banks).  Each event then costs a thread one LDS read
// and the comparisons in 32-bit arithmetic (every cumulative weight is below
// 2^32: the threshold planes are at most 32 and the largest total weight is
// below 2^B, or B < 32): about 60 instructions for 32 replicas per event,
// against about 750 for the bit-sliced word, so a word's chain of events
// finishes an order of magnitude sooner at about twice the work per
// replica-event: the choice for long chains on few replicas.
constexpr int kLanesRow = 36;                 // words per event row in sq
constexpr int kLanesHalfWords = 32 * kLanesRow;  // sq words per half wave

// In-register transpose of a 32 x 32 bit matrix: afterwards bit q of x[l] is
// bit l of the original x[q].  Five levels of block swaps (j = 16, 8, 4, 2,
// 1): the bits of row k at columns with bit j set trade places with those of
// row k + j at columns with bit j clear.
__device__ __forceinline__ void transpose32(uint32_t (&x)[32])
{
    constexpr uint32_t M[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int lv = 0; lv < 5; ++lv) {
        const int j = 16 >> lv;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (k & j) continue;
            const uint32_t t = ((x[k] >> j) ^ x[k + j]) & M[lv];
            x[k + j] ^= t;
            x[k] ^= t << j;
        }
    }
}

__device__ __forceinline__ void wm_lanes(const WmArgs &a, const uint64_t w, uint32_t *sq)
{
    if (w >= a.n_words) return;
    const int l = threadIdx.x & 31;
    const int hv = (threadIdx.x >> 5) & 1;
    const uint64_t i = 32 * w + (uint64_t)l;
    const bool live = i < a.M;
    const uint64_t E0 = live ? a.E[i] : 0, T0 = live ? a.Etgt[i] : 0;
    const bool mine = live && E0 < T0;
    // word window over pending lanes, as in wm_word
    uint64_t lo = mine ? E0 : ~0ull, hi = mine ? T0 : 0;
    for (int o = 16; o; o >>= 1) {
        const uint64_t lo2 = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)lo, o, 32) |
                             ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(lo >> 32), o, 32) << 32);
        const uint64_t hi2 = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)hi, o, 32) |
                             ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(hi >> 32), o, 32) << 32);
        lo = lo2 < lo ? lo2 : lo;
        hi = hi2 > hi ? hi2 : hi;
    }
    if (hi == 0) lo = hi = 0;
    if (a.max_events && hi > lo + a.max_events) hi = lo + a.max_events;

    const int nbm = a.nb_mem;
    int32_t cL = 0, cD = 0, cA = 0;
    for (int q = 0; q < nbm; ++q) {
        cL |= (int32_t)((a.planes[((uint64_t)0 * nbm + q) * a.wp + w] >> l) & 1u) << q;
        cD |= (int32_t)((a.planes[((uint64_t)1 * nbm + q) * a.wp + w] >> l) & 1u) << q;
        cA |= (int32_t)((a.planes[((uint64_t)2 * nbm + q) * a.wp + w] >> l) & 1u) << q;
    }
    const int B = a.B;  // at most 32 (the host's plane buckets)
    const uint64_t cu = a.cu;
    const bool has_a = a.fa >= 0, has_i = a.fi >= 0;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    uint32_t nreal = 0;
    // the reaction whose cumulative weight first exceeds n: with b_r = [n <
    // S_r] (monotone in r, S_1 = U, S_2 = 2U, ...), reaction r fires where
    // b_r and not b_(r-1); the count changes below are those of the five
    // reactions (A -> L, A -> D, A + L -> 2L, A + D -> 2D, L + D -> 2A)
    // summed over these indicators
    const uint32_t cu32 = (uint32_t)cu;
    const uint32_t amask = has_a ? ~0u : 0u, imask = has_i ? ~0u : 0u;
    const int fa = has_a ? a.fa : 0, fi = has_i ? a.fi : 0;
    auto apply = [&](uint32_t n, bool act) {
        const uint32_t A = (uint32_t)cA, L = (uint32_t)cL, D = (uint32_t)cD;
        const uint32_t U = cu32 * A;
        const uint32_t S2 = 2 * U;
        const uint32_t S3 = S2 + (((uint32_t)__umul24(A, L) & amask) << fa);
        const uint32_t S4 = S3 + (((uint32_t)__umul24(A, D) & amask) << fa);
        const uint32_t S5 = S4 + (((uint32_t)__umul24(L, D) & imask) << fi);
        const int32_t b0 = act && n < U, b1 = act && n < S2, b2 = act && n < S3;
        const int32_t b3 = act && n < S4, b4 = act && n < S5;
        cL += b0 - b1 + b2 + b3 - b4;
        cD += b1 - b0 - b2 + 2 * b3 - b4;
        cA += 2 * b4 - 3 * b3;
        nreal += (uint32_t)b4;
    };
    if (a.zs) {
        // shared threshold: the same n for every thread
        for (uint64_t e = lo; e < hi; ++e)
            apply(shared_at(a, e), mine && E0 <= e && e < T0);
    } else {
        const int nq = (B + 3) / 4;
        const uint32_t bmask = B >= 32 ? ~0u : ((1u << B) - 1u);
        for (uint64_t e0 = lo; e0 < hi; e0 += 32) {
            const uint64_t ed = e0 + (uint64_t)l;
            if (ed < hi) {
                uint32_t x[32];
#pragma unroll
                for (int q4 = 0; q4 < 8; ++q4) {
                    uint32_t o0 = 0, o1 = 0, o2 = 0, o3 = 0;
                    if (q4 < nq)
                        philox4x32_10((uint32_t)ed,
                                      (DOM_EVENT << 24) | ((uint32_t)q4 << 16) |
                                          ((uint32_t)(ed >> 32) & 0xFFFFu),
                                      (uint32_t)w, a.net_id, k0, k1, o0, o1, o2, o3);
                    x[4 * q4] = o0;
                    x[4 * q4 + 1] = o1;
                    x[4 * q4 + 2] = o2;
                    x[4 * q4 + 3] = o3;
                }
                transpose32(x);
                uint4 *row = reinterpret_cast<uint4 *>(sq + kLanesRow * l);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    row[c] = make_uint4(x[4 * c] & bmask, x[4 * c + 1] & bmask,
                                        x[4 * c + 2] & bmask, x[4 * c + 3] & bmask);
            }
            // the half's LDS operations run in program order: the reads below
            // see every lane's stores, and the next run's stores follow them
            __builtin_amdgcn_wave_barrier();
            const uint64_t left = hi - e0;
            const int gn = left < 32 ? (int)left : 32;
            for (int g = 0; g < gn; ++g) {
                const uint64_t e = e0 + (uint64_t)g;
                apply(sq[kLanesRow * g + l], mine && E0 <= e && e < T0);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    // pack the counts back into the planes of the word (lane 0 of the half stores)
    for (int q = 0; q < nbm; ++q) {
        const uint32_t bl = (uint32_t)(__ballot((cL >> q) & 1) >> (32 * hv));
        const uint32_t bd = (uint32_t)(__ballot((cD >> q) & 1) >> (32 * hv));
        const uint32_t ba = (uint32_t)(__ballot((cA >> q) & 1) >> (32 * hv));
        if (l == 0) {
            a.planes[((uint64_t)0 * nbm + q) * a.wp + w] = bl;
            a.planes[((uint64_t)1 * nbm + q) * a.wp + w] = bd;
            a.planes[((uint64_t)2 * nbm + q) * a.wp + w] = ba;
        }
    }
    if (live) a.E[i] = hi < E0 ? E0 : (hi > T0 ? T0 : hi);
    for (int o = 16; o; o >>= 1) nreal += (uint32_t)__shfl_xor((int)nreal, o, 32);
    if (l == 0) a.real[w] += nreal;
}

}  // namespace bwg
