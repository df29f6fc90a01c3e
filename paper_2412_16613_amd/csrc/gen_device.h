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

}  // namespace bwg
