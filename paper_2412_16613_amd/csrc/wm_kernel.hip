// Bit-parallel uniformised Gillespie step for Frank-family networks
// (well-mixed), one 32-bit word = 32 replicas per thread.
//
// What one event computes for every replica (lane) of a word, following the
// bitwise update of Sec. 4 of the paper:
//   (a) a uniform threshold n on [0, 2^B), one bit plane per random word
//       (per-replica draws instead of the paper's shared n, Sec. 4 step a);
//   (b)-(d) the comparator/changer construction: with cumulative weights
//       S_1..S_5 of the reactions A->L, A->D, A+L->2L, A+D->2D, L+D->2A the
//       changer of reaction r is [n < S_r] & ~[n < S_{r-1}] (Eq. (24) with
//       omega = [m <= n] of the previous reaction); a lane with no changer
//       set takes the null event (ghost reactions, Eqs. (4)-(6), (9));
//   (e) the occupancy update N += xi & nu_r (Eq. (27)) as masked ripple-carry
//       increments and decrements (Sec. 4.1.1);
//   (f) the incremental product update of App. B: with masked occupancies and
//       only additions, subtractions and doublings, never a product of two
//       occupancies (Eqs. (B.1)-(B.3), Sec. 4.1.2).
//
// The cumulative weights are S_1 = U, S_2 = 2U, S_3 = 2U + 2^fa P_AL,
// S_4 = S_3 + 2^fa P_AD, S_5 = S_4 + 2^fi P_LD with U = cu N_A and the pair
// counts P_XY = N_X N_Y.  The comparisons against S_3..S_5 are done as one
// borrow chain per reaction on d = n - 2U - ..., so each reaction costs one
// subtraction instead of an addition plus a comparison.
//
// Products are updated with  X'Y' - XY = dX * Y' + dY * X  (X before, Y after
// the event), a sum of two masked, possibly negated or doubled, occupancies
// formed in NB+2 planes and added sign-extended to the product.

#include "wm_device.h"

namespace bwg {

template <int NB, int BC, int FA, int CU, bool SH, int NT, int BS>
__global__ __launch_bounds__(256) void wm_event_kernel(WmArgs a)
{
    wm_word<NB, BC, FA, CU, SH, FA, NT, BS>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Producer/consumer form: four waves per 128 words, events handed over
// through two rings of 2 x PH events of threshold planes in LDS (PH x BC KiB
// in all, at most 128 KiB: the form runs at most 256 workgroups, one per
// CU).  PH as measured best on the named workloads (3, 4, 6 and 8 tried).
template <int BC>
constexpr int pc_half()
{
    return BC == 20 ? 6 : 4;
}

template <int NB, int BC, int FA, int CU, int NT, int BS>
__global__ __launch_bounds__(256) void wm_pc_kernel(WmArgs a)
{
    constexpr int PH = pc_half<BC>();
    __shared__ uint4 ring[2 * 2 * PH][BC / 4][64];
    __shared__ uint64_t wave_span[4];
    wm_word_pc<NB, BC, FA, CU, PH, FA, NT, BS>(a, ring, wave_span);
}

// Other word widths (16 or 64 replicas per thread), one wave per 64 threads.
template <int NB, int BC, int FA, int CU, bool SH, int NT, int BS, int WW>
__global__ __launch_bounds__(256) void wm_event_w_kernel(WmArgs a)
{
    wm_word_w<NB, BC, FA, CU, SH, FA, NT, BS, WW>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <int NB, int BC, int FA, int CU, int NT, int BS, int WW>
hipError_t launch_wm_w(const WmArgs &a, hipStream_t s, int block)
{
    const uint64_t threads = WW == 64 ? (a.n_words + 1) / 2 : 2 * a.n_words;
    if (block <= 0) block = threads >= 65536 ? 256 : 128;
    const uint64_t grid = (threads + block - 1) / block;
    if (a.zs)
        hipLaunchKernelGGL((wm_event_w_kernel<NB, BC, FA, CU, true, NT, BS, WW>),
                           dim3((uint32_t)grid), dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL((wm_event_w_kernel<NB, BC, FA, CU, false, NT, BS, WW>),
                           dim3((uint32_t)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

template <int NB, int BC, int FA, int CU, int NT, int BS>
hipError_t launch_wm(const WmArgs &a, hipStream_t s, int block, int word_bits)
{
    if (word_bits == 16 || word_bits == 64) {
        // compile-time weights only (the host checks before any launch)
        if constexpr (FA >= 0 && CU >= 0) {
            return word_bits == 16 ? launch_wm_w<NB, BC, FA, CU, NT, BS, 16>(a, s, block)
                                   : launch_wm_w<NB, BC, FA, CU, NT, BS, 64>(a, s, block);
        } else {
            return hipErrorInvalidValue;
        }
    }
    // with at most one wave of 64 words per SIMD pair half the chip would
    // idle: split each word's events over a producer and a consumer wave
    if (block <= 0 && !a.zs && a.n_words <= 32768) {
        hipLaunchKernelGGL((wm_pc_kernel<NB, BC, FA, CU, NT, BS>), dim3((uint32_t)((a.n_words + 127) / 128)),
                           dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // 128-thread blocks leave two SIMDs of a CU to other blocks, which pays
    // while there are fewer words than one wave per SIMD; from 1024 waves on,
    // 256-thread blocks (one wave per SIMD of a CU) keep the waves spread
    // evenly when the occupancy would let some CUs take more than their share
    if (block <= 0) block = a.n_words >= 65536 ? 256 : 128;
    const uint64_t grid = (a.n_words + block - 1) / block;
    if (a.zs)
        hipLaunchKernelGGL((wm_event_kernel<NB, BC, FA, CU, true, NT, BS>), dim3((uint32_t)grid),
                           dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL((wm_event_kernel<NB, BC, FA, CU, false, NT, BS>), dim3((uint32_t)grid),
                           dim3(block), 0, s, a);
    return hipGetLastError();
}

// Kernel instantiations (both compilation passes) and the host-side table.
// (NB, BC, FA, CU, NT, BS): FA/CU = -1 are taken at run time; NT > 0 fixes
// the molecule count and BS the selection planes (exact register widths,
// see WmShape), NT = 0 serves any count within the planes.
#define BWG_WM_VARIANTS(X) BWG_WM_VARIANTS_CT(X) BWG_WM_VARIANTS_RT(X)
#define BWG_WM_VARIANTS_CT(X)                                                 \
    /* the named workloads, exact widths */                                   \
    X(6, 20, 9, 164, 32, 18)     /* N_tot = 32, k0 = 0.01, k1 = k2 = 1/32 */  \
    X(11, 24, 4, 164, 1024, 23)  /* N_tot = 1024 */                           \
    /* the paper's network (unit weights, no conversions) by N_tot */        \
    X(4, 8, 0, 0, 0, 8)      /* N_tot <= 15 */                                \
    X(5, 8, 0, 0, 0, 8)      /* N_tot <= 23 */                                \
    X(6, 12, 0, 0, 0, 12)    /* N_tot <= 63 */                                \
    X(7, 12, 0, 0, 0, 12)    /* N_tot <= 91 */                                \
    X(8, 16, 0, 0, 0, 16)    /* N_tot <= 255 */                               \
    X(9, 16, 0, 0, 0, 16)    /* N_tot <= 362 */                               \
    X(10, 20, 0, 0, 0, 20)   /* N_tot <= 1023 */                              \
    X(11, 20, 0, 0, 0, 20)   /* N_tot <= 1448 */
#define BWG_WM_VARIANTS_RT(X)                                                 \
    /* run-time shifts and weights, any Frank-family network in budget */     \
    X(4, 20, -1, -1, 0, 20)                                                   \
    X(6, 20, -1, -1, 0, 20)                                                   \
    X(8, 24, -1, -1, 0, 24)                                                   \
    X(10, 24, -1, -1, 0, 24)                                                  \
    X(12, 28, -1, -1, 0, 28)                                                  \
    X(14, 32, -1, -1, 0, 32)

// Lanes engine: 8 words per 256-thread block, one replica per thread; the
// launch's piece starts at word w0.
__global__ __launch_bounds__(256) void wm_lanes_kernel(WmArgs a, uint64_t w0)
{
    __shared__ __align__(16) uint32_t sq[8][kLanesHalfWords];
    const int half = threadIdx.x >> 5;
    wm_lanes(a, w0 + 8 * (uint64_t)blockIdx.x + half, sq[half]);
}

// Shared thresholds of events e0 .. e0 + len - 1, one thread per event.
__global__ __launch_bounds__(256) void shared_fill_kernel(uint32_t *tab, uint64_t e0, uint64_t len,
                                                          uint64_t seed, uint32_t net_id, uint32_t Z,
                                                          uint64_t k0)
{
    const uint64_t k = k0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) tab[k] = shared_threshold(seed, net_id, e0 + k, Z, (0u - Z) % Z);
}

hipError_t launch_shared_fill(uint32_t *tab, uint64_t e0, uint64_t len, uint64_t seed,
                              uint32_t net_id, uint32_t Z, hipStream_t s)
{
    return launch_pieces(len, 256, [&](uint64_t k0, dim3 g) {
        hipLaunchKernelGGL(shared_fill_kernel, g, dim3(256), 0, s, tab, e0, len, seed, net_id, Z,
                           k0);
    });
}

hipError_t launch_wm_lanes(const WmArgs &a, hipStream_t s)
{
    // one work-item per replica slot: pieces of kLaunchSpan / 32 words
    return launch_pieces(32 * a.n_words, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(wm_lanes_kernel, g, dim3(256), 0, s, a, i0 / 32);
    });
}

#define BWG_WM_INST(nb, bc, fa, cu, nt, bs)                                     \
    template __global__ void wm_event_kernel<nb, bc, fa, cu, false, nt, bs>(WmArgs); \
    template __global__ void wm_event_kernel<nb, bc, fa, cu, true, nt, bs>(WmArgs);  \
    template __global__ void wm_pc_kernel<nb, bc, fa, cu, nt, bs>(WmArgs);
BWG_WM_VARIANTS(BWG_WM_INST)

// 16 and 64 replicas per thread for the compile-time variants
#define BWG_WM_INST_W(nb, bc, fa, cu, nt, bs)                                         \
    template __global__ void wm_event_w_kernel<nb, bc, fa, cu, false, nt, bs, 16>(WmArgs); \
    template __global__ void wm_event_w_kernel<nb, bc, fa, cu, true, nt, bs, 16>(WmArgs);  \
    template __global__ void wm_event_w_kernel<nb, bc, fa, cu, false, nt, bs, 64>(WmArgs); \
    template __global__ void wm_event_w_kernel<nb, bc, fa, cu, true, nt, bs, 64>(WmArgs);
BWG_WM_VARIANTS_CT(BWG_WM_INST_W)

#ifndef __HIP_DEVICE_COMPILE__
#define BWG_WM_ENTRY(nb, bc, fa, cu, nt, bs) {nb, bc, fa, cu, nt, bs, &launch_wm<nb, bc, fa, cu, nt, bs>},
const WmVariant kWmVariants[] = {BWG_WM_VARIANTS(BWG_WM_ENTRY)};
const int kWmVariantCount = sizeof(kWmVariants) / sizeof(kWmVariants[0]);
#endif

}  // namespace bwg
