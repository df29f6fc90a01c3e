// Device helpers: 3-input bitwise operations, Philox4x32-10, bit-sliced
// ripple arithmetic on arrays of bit planes (plane q holds bit q of 32
// replicas, one per bit lane).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bwg {

// v_bitop3_b32 computes an arbitrary 3-input function given by its truth
// table over (src0, src1, src2) = (0xF0, 0xCC, 0xAA).
constexpr uint32_t TA = 0xF0, TB = 0xCC, TC = 0xAA;
constexpr uint32_t lut(uint32_t v) { return v & 0xFFu; }

constexpr uint32_t L_XOR3 = lut(TA ^ TB ^ TC);                        // sum bit
constexpr uint32_t L_MAJ = lut((TA & TB) | (TA & TC) | (TB & TC));    // carry of a+b+c
constexpr uint32_t L_BORROW = lut((~TA & TB) | (~TA & TC) | (TB & TC));  // borrow of a-b-c
constexpr uint32_t L_ANDXOR = lut((TA & TB) ^ TC);                    // (a & b) ^ c
constexpr uint32_t L_ANDOR = lut((TA & TB) | TC);                     // (a & b) | c
constexpr uint32_t L_ANDNOT = lut(TA & ~TB);                          // a & ~b (c unused)
constexpr uint32_t L_ANDNOT_OR = lut((TA & ~TB) | TC);                // (a & ~b) | c

#define BWG_OP3(a, b, c, L) __builtin_amdgcn_bitop3_b32((a), (b), (c), (L))

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -------------------
// Ten rounds of: multiply counter words 0 and 2 by the two Philox constants;
// new counter = (hi(w2*M1) ^ w1 ^ k0, lo(w2*M1), hi(w0*M0) ^ w3 ^ k1,
// lo(w0*M0)); the key advances by the two Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t k0, uint32_t k1,
                                              uint32_t &o0, uint32_t &o1, uint32_t &o2,
                                              uint32_t &o3)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // one 3-input xor each (the round key is wave-uniform)
        const uint32_t n0 = BWG_OP3((uint32_t)(p1 >> 32), c1, k0, L_XOR3);
        const uint32_t n2 = BWG_OP3((uint32_t)(p0 >> 32), c3, k1, L_XOR3);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    o0 = c0;
    o1 = c1;
    o2 = c2;
    o3 = c3;
}

// ---- bit-sliced arithmetic ------------------------------------------------
// Planes are uint32 arrays, least significant plane first.  All operations
// are modulo 2^width of the destination.  The in-place ripple updates form
// each plane's carry before overwriting the plane, so the new value can take
// the old one's register (in an event loop, no copies at the loop latch).

// Masked increment/decrement/double by per-lane masks: x += d with
// d = +1 on `plus`, -1 on `minus`, 0 elsewhere (plus & minus = 0).
template <int W>
__device__ __forceinline__ void add_pm1(uint32_t (&x)[W], uint32_t plus, uint32_t minus)
{
    // two's complement addend: plane 0 = plus | minus, planes >= 1 = minus
    uint32_t c = x[0] & (plus | minus);
    x[0] ^= (plus | minus);
#pragma unroll
    for (int q = 1; q < W; ++q) {
        const uint32_t cn = q + 1 < W ? BWG_OP3(x[q], minus, c, L_MAJ) : 0u;
        x[q] = BWG_OP3(x[q], minus, c, L_XOR3);
        c = cn;
    }
}

// x += d with d = -1 on `minus1`, +2 on `plus2`, 0 elsewhere (disjoint).
template <int W>
__device__ __forceinline__ void add_m1_p2(uint32_t (&x)[W], uint32_t minus1, uint32_t plus2)
{
    // addend planes: q = 0: minus1; q = 1: minus1 | plus2; q >= 2: minus1
    uint32_t c = x[0] & minus1;
    x[0] ^= minus1;
    if (W > 1) {
        const uint32_t a1 = minus1 | plus2;
        const uint32_t cn = BWG_OP3(x[1], a1, c, L_MAJ);
        x[1] = BWG_OP3(x[1], a1, c, L_XOR3);
        c = cn;
    }
#pragma unroll
    for (int q = 2; q < W; ++q) {
        const uint32_t cn = q + 1 < W ? BWG_OP3(x[q], minus1, c, L_MAJ) : 0u;
        x[q] = BWG_OP3(x[q], minus1, c, L_XOR3);
        c = cn;
    }
}

// acc (WA planes) += sign-extended d (WD planes) + carry_in.
template <int WA, int WD>
__device__ __forceinline__ void add_sext(uint32_t (&acc)[WA], const uint32_t (&d)[WD],
                                         uint32_t carry_in)
{
    uint32_t c = carry_in;
    const uint32_t sgn = d[WD - 1];
#pragma unroll
    for (int q = 0; q < WA; ++q) {
        const uint32_t v = q < WD ? d[q] : sgn;
        const uint32_t cn = q + 1 < WA ? BWG_OP3(acc[q], v, c, L_MAJ) : 0u;
        acc[q] = BWG_OP3(acc[q], v, c, L_XOR3);
        c = cn;
    }
}

// Bit-sliced product of two NB-plane numbers into WP planes (schoolbook).
template <int NB, int WP>
__device__ __forceinline__ void mul_planes(uint32_t (&out)[WP], const uint32_t (&x)[NB],
                                           const uint32_t (&y)[NB])
{
#pragma unroll
    for (int q = 0; q < WP; ++q) out[q] = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        uint32_t c = 0;
#pragma unroll
        for (int q = j; q < WP; ++q) {
            const uint32_t v = (q - j < NB) ? (x[q - j] & y[j]) : 0u;
            const uint32_t s = BWG_OP3(out[q], v, c, L_XOR3);
            c = BWG_OP3(out[q], v, c, L_MAJ);
            out[q] = s;
        }
    }
}

}  // namespace bwg
