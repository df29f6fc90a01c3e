// Device self-test of the bit-sliced primitives (bitops.h, wm_device.h):
// every primitive runs on GPU words built from all operand combinations of a
// small width, and the per-lane results come back as integers for the tests
// to compare with integer arithmetic.  Test infrastructure: the library's
// kernels do not use this file.
//
// Combination k is lane k mod 32 of word k / 32; each thread packs its
// word's 32 combinations into bit planes, applies the primitive and unpacks.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wm_device.h"

namespace {

using namespace bwg;

// planes of the values v(l), l < 32 (plane q holds bit q of lane l)
template <int W, class F>
__device__ void pack(uint32_t (&p)[W], F v)
{
#pragma unroll
    for (int q = 0; q < W; ++q) p[q] = 0;
    for (int l = 0; l < 32; ++l) {
        const uint32_t x = v(l);
#pragma unroll
        for (int q = 0; q < W; ++q) p[q] |= ((x >> q) & 1u) << l;
    }
}

template <int W>
__device__ uint32_t lane_value(const uint32_t (&p)[W], int l)
{
    uint32_t x = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) x |= ((p[q] >> l) & 1u) << q;
    return x;
}

// op 0: add_pm1<6>: x = k % 64, d = k / 64 in {0: +1, 1: -1, 2: 0}
// op 1: add_m1_p2<6>: x = k % 64, d = k / 64 in {0: -1, 1: +2, 2: 0}
// op 2: add_sext<10, 6>: acc = k % 1024, d = (k / 1024) % 64 as 6-bit two's
//       complement, carry-in = k / 65536
// op 3: mul_planes<6, 10>: x = k % 64, y = k / 64
// op 4: sub_shifted<2, 12, 6, KEEP, 12>: d = k % 4096, p = k / 4096 (< 64);
//       out = difference mod 2^12 | borrow << 12
// op 5: sub_shifted<3, 12, 6, no keep, 10> borrow of planes [3, 10) only:
//       d = k % 1024, p = k / 1024 (< 64); out = borrow
__global__ void prim_kernel(int op, uint32_t n_combos, uint32_t *out)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (32 * w >= n_combos) return;
    const uint32_t k0 = 32 * w;
    uint32_t res[32];
    if (op == 0 || op == 1) {
        uint32_t x[6];
        pack<6>(x, [&](int l) { return (k0 + l) % 64u; });
        uint32_t m0 = 0, m1 = 0;
        for (int l = 0; l < 32; ++l) {
            const uint32_t d = (k0 + l) / 64u;
            m0 |= (d == 0 ? 1u : 0u) << l;
            m1 |= (d == 1 ? 1u : 0u) << l;
        }
        if (op == 0)
            add_pm1<6>(x, m0, m1);
        else
            add_m1_p2<6>(x, m0, m1);
        for (int l = 0; l < 32; ++l) res[l] = lane_value<6>(x, l);
    } else if (op == 2) {
        uint32_t acc[10], d[6], cin = 0;
        pack<10>(acc, [&](int l) { return (k0 + l) % 1024u; });
        pack<6>(d, [&](int l) { return ((k0 + l) / 1024u) % 64u; });
        for (int l = 0; l < 32; ++l) cin |= (((k0 + l) / 65536u) & 1u) << l;
        add_sext<10, 6>(acc, d, cin);
        for (int l = 0; l < 32; ++l) res[l] = lane_value<10>(acc, l);
    } else if (op == 3) {
        uint32_t x[6], y[6], p[10];
        pack<6>(x, [&](int l) { return (k0 + l) % 64u; });
        pack<6>(y, [&](int l) { return (k0 + l) / 64u; });
        mul_planes<6, 10>(p, x, y);
        for (int l = 0; l < 32; ++l) res[l] = lane_value<10>(p, l);
    } else if (op == 4) {
        uint32_t d[12], p[6];
        pack<12>(d, [&](int l) { return (k0 + l) % 4096u; });
        pack<6>(p, [&](int l) { return (k0 + l) / 4096u; });
        const uint32_t br = sub_shifted<2, 12, 6, true, 12>(d, p);
        for (int l = 0; l < 32; ++l) res[l] = lane_value<12>(d, l) | (((br >> l) & 1u) << 12);
    } else {
        uint32_t d[12], p[6];
        pack<12>(d, [&](int l) { return (k0 + l) % 1024u; });
        pack<6>(p, [&](int l) { return (k0 + l) / 1024u; });
        const uint32_t br = sub_shifted<3, 12, 6, false, 10>(d, p);
        for (int l = 0; l < 32; ++l) res[l] = (br >> l) & 1u;
    }
    for (int l = 0; l < 32; ++l)
        if (k0 + l < n_combos) out[k0 + l] = res[l];
}

}  // namespace

// Run primitive `op` over n_combos combinations into out (device, n_combos
// uint32) on `stream`; 0 or the HIP error code.
extern "C" int bwg_selftest_prim(int op, uint32_t n_combos, uint32_t *out, void *stream)
{
    const uint32_t words = (n_combos + 31) / 32;
    hipLaunchKernelGGL(prim_kernel, dim3((words + 63) / 64), dim3(64), 0, (hipStream_t)stream, op,
                       n_combos, out);
    return (int)hipGetLastError();
}
