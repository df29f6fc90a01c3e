// Comparator engine: the same uniformised chain with one replica per thread
// and int32 counts -- the standard Gillespie iteration of Sec. 3 of the
// paper (draw n, evaluate the weights, linear CDF search, apply nu_r), run
// for many replicas in parallel the way a plain GPU SSA would.  It has its
// own random stream (PLAIN domain): the threshold of event e of replica i is
// the low B bits of output (e mod 4) of the Philox call keyed by e/4.

#include "bitops.h"
#include "bwg_internal.h"

namespace bwg {

__global__ __launch_bounds__(256) void plain_event_kernel(PlainArgs a, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.M) return;
    int32_t N[3] = {a.counts[3 * i], a.counts[3 * i + 1], a.counts[3 * i + 2]};
    const uint64_t e0 = a.E[i];
    uint64_t e1 = a.Etgt[i];
    if (a.max_events && e1 > e0 + a.max_events) e1 = e0 + a.max_events;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const uint32_t bmask = a.B >= 32 ? 0xFFFFFFFFu : ((1u << a.B) - 1u);
    uint32_t o[4] = {0, 0, 0, 0};
    uint64_t nreal = 0;
    for (uint64_t e = e0; e < e1; ++e) {
        if (e == e0 || (e & 3u) == 0) {
            const uint64_t blk = e >> 2;
            philox4x32_10((uint32_t)blk, (DOM_PLAIN << 24) | ((uint32_t)(blk >> 32) & 0xFFFFu),
                          (uint32_t)i, a.net_id, k0, k1, o[0], o[1], o[2], o[3]);
        }
        const uint32_t sel = (uint32_t)(e & 3u);
        const uint32_t r32 = sel == 0 ? o[0] : sel == 1 ? o[1] : sel == 2 ? o[2] : o[3];
        const uint64_t n = r32 & bmask;
        uint64_t m = 0;
        int r = -1;
        for (int j = 0; j < a.R; ++j) {
            const PlainReaction &rx = a.rx[j];
            const int32_t nx = rx.x == 0 ? N[0] : rx.x == 1 ? N[1] : N[2];
            const int32_t ny = rx.y == 0 ? N[0] : rx.y == 1 ? N[1] : N[2];
            uint64_t h;
            if (rx.kind == 0)
                h = (uint64_t)nx;
            else if (rx.kind == 1)
                h = (uint64_t)nx * (uint64_t)ny;
            else
                h = (uint64_t)nx * (uint64_t)(nx > 0 ? nx - 1 : 0) / 2;
            m += (uint64_t)rx.c * h;
            if (r < 0 && n < m) r = j;
        }
        if (r >= 0) {
            const PlainReaction &rx = a.rx[r];
            N[0] += rx.d[0];
            N[1] += rx.d[1];
            N[2] += rx.d[2];
            nreal += (rx.d[0] | rx.d[1] | rx.d[2]) != 0;
        }
    }
    a.counts[3 * i] = N[0];
    a.counts[3 * i + 1] = N[1];
    a.counts[3 * i + 2] = N[2];
    a.E[i] = e1;
    a.real[i] += nreal;
}

hipError_t launch_plain(const PlainArgs &a, hipStream_t s, int block)
{
    if (block <= 0) block = 256;
    return launch_pieces(a.M, (uint32_t)block, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(plain_event_kernel, g, dim3(block), 0, s, a, i0);
    });
}

// Initial state of the plain engine: fixed counts or the multinomial draw
// (same INIT contract as the bit-sliced engine).
__global__ void plain_init_kernel(int32_t *counts, uint64_t M, int mode, int32_t c0, int32_t c1,
                                  int32_t c2, int64_t n_tot, uint64_t seed, uint32_t net_id,
                                  uint64_t *E, uint64_t *Et, uint64_t *real, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    if (mode == 0) {
        counts[3 * i] = c0;
        counts[3 * i + 1] = c1;
        counts[3 * i + 2] = c2;
    } else {
        int32_t nL = 0, nD = 0, nA = 0;
        uint32_t o[4] = {0, 0, 0, 0};
        for (int64_t m = 0; m < n_tot; ++m) {
            if ((m & 63) == 0)
                philox4x32_10((uint32_t)(m >> 6), DOM_INIT << 24, (uint32_t)i, net_id,
                              (uint32_t)seed, (uint32_t)(seed >> 32), o[0], o[1], o[2], o[3]);
            const int bit = (int)(2 * (m & 63));
            const uint32_t v = (o[bit >> 5] >> (bit & 31)) & 3u;
            nL += v == 0;
            nD += v == 1;
            nA += v >= 2;
        }
        counts[3 * i] = nL;
        counts[3 * i + 1] = nD;
        counts[3 * i + 2] = nA;
    }
    E[i] = 0;
    Et[i] = 0;
    real[i] = 0;
}

hipError_t launch_plain_init(int32_t *counts, uint64_t M, int mode, const int32_t c[3],
                             int64_t n_tot, uint64_t seed, uint32_t net_id, uint64_t *E,
                             uint64_t *Et, uint64_t *real, hipStream_t s)
{
    return launch_pieces(M, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(plain_init_kernel, g, dim3(256), 0, s, counts, M, mode, c[0], c[1],
                           c[2], n_tot, seed, net_id, E, Et, real, i0);
    });
}

}  // namespace bwg
