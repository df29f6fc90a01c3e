// Bit-parallel uniformised Gillespie step for any 3-species network of
// order <= 2 (the method of Sec. 4 with the weights of Eq. (7) computed from
// the bit planes at every event instead of the Frank-specific incremental
// products).  One thread per word of 32 replicas; per event:
//   (a) threshold planes n from the same EVENT draws as the Frank kernel;
//   (b) the weight kinds some reaction uses, from the occupancies: N_X as
//       it is, pair counts N_X N_Y and N_X (N_X - 1) / 2 by bit-sliced
//       schoolbook products, each kept in this thread's slot of LDS;
//   (c) first crossing in table order: d = n, and for each reaction j and
//       each set bit k of its integer weight c_j, d -= h_j << k; a lane
//       whose subtraction borrows has n < S_j (the borrow stays set for
//       the later reactions), so xi_j = [n < S_j] & ~[n < S_{j-1}];
//   (d) occupancies N_X += sum_j nu_jX xi_j as one masked add of a
//       constant in {-2..2} per species.

#include "gen_device.h"

namespace bwg {

template <int NB, int BC>
__global__ __launch_bounds__(64) void gen_event_kernel(WmArgs a, GenNet g)
{
    static_assert(BC % 4 == 0, "threshold planes come in Philox quads");
    constexpr int WH = 2 * NB;  // planes of a pair count
    extern __shared__ uint32_t hs[];  // [slot][WH][64]
    const int tid = threadIdx.x;
    const uint64_t w = (uint64_t)blockIdx.x * 64 + tid;
    if (w >= a.n_words) return;
    const uint32_t live = live_lanes(a, w);
    const uint64_t *E = a.E + 32 * w;
    const uint64_t *T = a.Etgt + 32 * w;
    const WordWindow win = word_window(a, E, T, live);
    uint32_t N[3][NB];
    load_word<NB>(a, w, N[0], N[1], N[2]);
    if (win.lo < win.hi) {
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const int nq = (a.B + 3) / 4;
        uint32_t lastm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) lastm[j] = (4 * (nq - 1) + j < a.B) ? ~0u : 0u;
        uint64_t nreal = 0;
        uint64_t nxt = 0;  // next event at which the active lanes change
        uint32_t actc = 0;
        for (uint64_t e = win.lo; e < win.hi; ++e) {
            if (e >= nxt) actc = lane_mask_next(E, T, win.pend, e, win.blo, nxt);
            const uint32_t act = actc;
            // (b) weight kinds into LDS
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                if (!((g.used >> k) & 1u)) continue;
                uint32_t h[WH];
                if (k < 3) {
#pragma unroll
                    for (int q = 0; q < WH; ++q) h[q] = q < NB ? N[k][q] : 0u;
                } else if (k < 6) {
                    constexpr int PX[3] = {0, 0, 1}, PY[3] = {1, 2, 2};
                    mul_planes<NB, WH>(h, N[PX[k - 3]], N[PY[k - 3]]);
                } else {
                    // X (X - 1) / 2: the product with X - 1 (all ones where
                    // X = 0, giving 0), then one plane down
                    uint32_t xm[NB];
#pragma unroll
                    for (int q = 0; q < NB; ++q) xm[q] = N[k - 6][q];
                    add_pm1<NB>(xm, 0u, ~0u);
                    uint32_t p[WH];
                    mul_planes<NB, WH>(p, N[k - 6], xm);
#pragma unroll
                    for (int q = 0; q < WH; ++q) h[q] = q + 1 < WH ? p[q + 1] : 0u;
                }
                uint32_t *dst = hs + (uint32_t)g.slot[k] * WH * 64 + tid;
#pragma unroll
                for (int q = 0; q < WH; ++q) dst[q * 64] = h[q];
            }
            // (a) thresholds, (c) first crossing in table order
            uint32_t d[BC];
            philox_planes<BC>(d, e, (uint32_t)w, a.net_id, k0, k1, nq, lastm);
            uint32_t lt = 0, realm = 0;
            uint32_t m[3][4] = {};  // per species: +1, -1, +2, -2
            for (int j = 0; j < g.R; ++j) {
                const uint32_t *src = hs + (uint32_t)g.slot[g.kind[j]] * WH * 64 + tid;
                uint32_t h[WH];
#pragma unroll
                for (int q = 0; q < WH; ++q) h[q] = src[q * 64];
                uint32_t br = 0;
                for (uint32_t c = g.c[j]; c; c &= c - 1)
                    br |= sub_dispatch<BC, WH, true>(__builtin_ctz(c), d, h);
                const uint32_t ltj = lt | br;
                const uint32_t xi = ltj & ~lt & act;
                lt = ltj;
                if ((g.change >> j) & 1u) realm |= xi;
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const int dv = g.d[j][x];
                    m[x][0] |= dv == 1 ? xi : 0u;
                    m[x][1] |= dv == -1 ? xi : 0u;
                    m[x][2] |= dv == 2 ? xi : 0u;
                    m[x][3] |= dv == -2 ? xi : 0u;
                }
            }
            nreal += (uint32_t)__builtin_popcount(realm);
            // (d) occupancies
#pragma unroll
            for (int x = 0; x < 3; ++x) add_delta<NB>(N[x], m[x][0], m[x][1], m[x][2], m[x][3]);
        }
        a.real[w] += nreal;
    }
    store_word<NB>(a, w, live, win.hi, N[0], N[1], N[2]);
}

template <int NB, int BC>
hipError_t launch_gen(const WmArgs &a, const GenNet &g, hipStream_t s)
{
    const size_t lds = (size_t)(g.n_slots > 0 ? g.n_slots : 1) * 2 * NB * 64 * sizeof(uint32_t);
    hipLaunchKernelGGL((gen_event_kernel<NB, BC>), dim3((uint32_t)((a.n_words + 63) / 64)),
                       dim3(64), lds, s, a, g);
    return hipGetLastError();
}

// (NB, BC) instantiations: count planes and threshold-plane capacity.
#define BWG_GEN_VARIANTS(X) \
    X(4, 12)                \
    X(6, 16)                \
    X(8, 20)                \
    X(11, 24)               \
    X(14, 32)

#define BWG_GEN_INST(nb, bc) template __global__ void gen_event_kernel<nb, bc>(WmArgs, GenNet);
BWG_GEN_VARIANTS(BWG_GEN_INST)

#ifndef __HIP_DEVICE_COMPILE__
#define BWG_GEN_ENTRY(nb, bc) {nb, bc, &launch_gen<nb, bc>},
const GenVariant kGenVariants[] = {BWG_GEN_VARIANTS(BWG_GEN_ENTRY)};
const int kGenVariantCount = sizeof(kGenVariants) / sizeof(kGenVariants[0]);
#endif

}  // namespace bwg
