// Issue-rate reference kernels for the VALU roofline: how many 32-bit lane
// operations per second the chip sustains for the instruction the bit-sliced
// kernels are made of (v_bitop3_b32, one 3-input LUT per 32 lanes of
// replicas) and for the 32 x 32 -> 64 bit multiply-add of Philox
// (v_mad_u64_u32), at a chosen number of waves per SIMD.  Measurement only:
// nothing of the simulation runs here.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;  // independent dependency chains per thread

// Every thread runs `iters` rounds of 16 x kChains bitop3 instructions in
// CH independent chains (full-adder sum LUT, so nothing folds; CH = 1 is
// one fully dependent chain, which measures the dependent-issue latency)
// and writes their xor at the end.
template <int CH>
__global__ __launch_bounds__(256) void bitop3_issue_kernel(uint32_t *out, uint32_t seed,
                                                          uint32_t iters)
{
    static_assert(kChains % CH == 0, "chains");
    uint32_t v[kChains];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = t * 0x9E3779B9u + c * 0x85EBCA6Bu + seed;
    // a and b are wave-uniform (scalar operands): the loop issues nothing but
    // the bitop3 chains and the loop counter
    uint32_t a = seed, b = ~seed;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                v[c % CH] = __builtin_amdgcn_bitop3_b32(v[c % CH], a + k + c, b, 0x96);
        }
        a += 0x9E3779B9u;
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= v[c];
    out[t] = r;
}

// The same with v_mad_u64_u32: 64-bit accumulators updated by 32 x 32
// products (Philox's round multiply is one such instruction).
__global__ __launch_bounds__(256) void mad64_issue_kernel(uint32_t *out, uint32_t seed,
                                                         uint32_t iters)
{
    uint64_t v[kChains];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = (uint64_t)(t * 0x9E3779B9u + c) << 7 | seed;
    const uint32_t m = 0xD2511F53u ^ seed;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) v[c] = (uint64_t)(uint32_t)v[c] * m + v[c];
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= (uint32_t)v[c] ^ (uint32_t)(v[c] >> 32);
    out[t] = r;
}

// Two-operand 32-bit adds (v_add_u32 of two registers), the kind of
// instruction the lanes engine is mostly made of: in each step every one of
// kChains accumulators adds its neighbour's value, so the adds stay
// separate instructions with kChains of them independent at a time.  Each
// step counts kChains instructions.
__global__ __launch_bounds__(256) void add_issue_kernel(uint32_t *out, uint32_t seed,
                                                       uint32_t iters)
{
    uint32_t v[kChains];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = t * 0x9E3779B9u + c * 0x85EBCA6Bu + seed;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                // written out so the compiler cannot merge two adds into v_add3_u32
                asm volatile("v_add_u32_e32 %0, %0, %1" : "+v"(v[c]) : "v"(v[(c + 1 + k) % kChains]));
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= v[c];
    out[t] = r;
}

}  // namespace

// Run one reference kernel: kind 0 = bitop3 (8 chains), 1 = mad_u64 (8
// chains), 2 = bitop3 (1 chain), 3 = bitop3 (2 chains), 4 = v_add_u32 (8
// accumulators); `blocks` blocks of
// 256 threads (4 waves), each thread 16 * kChains * iters instructions of
// that kind; out holds blocks * 256 uint32.  Returns the kernel's duration
// in ms (HIP events on `stream`), or a negative value on a HIP error.
extern "C" double bwg_valu_ref(int kind, uint32_t blocks, uint32_t iters, uint32_t *out,
                               void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
    hipEventRecord(a, s);
    if (kind == 0)
        hipLaunchKernelGGL(bitop3_issue_kernel<8>, dim3(blocks), dim3(256), 0, s, out, 1u, iters);
    else if (kind == 1)
        hipLaunchKernelGGL(mad64_issue_kernel, dim3(blocks), dim3(256), 0, s, out, 1u, iters);
    else if (kind == 2)
        hipLaunchKernelGGL(bitop3_issue_kernel<1>, dim3(blocks), dim3(256), 0, s, out, 1u, iters);
    else if (kind == 3)
        hipLaunchKernelGGL(bitop3_issue_kernel<2>, dim3(blocks), dim3(256), 0, s, out, 1u, iters);
    else
        hipLaunchKernelGGL(add_issue_kernel, dim3(blocks), dim3(256), 0, s, out, 1u, iters);
    const hipError_t le = hipGetLastError();
    hipEventRecord(b, s);
    float ms = -1.0f;
    if (le == hipSuccess && hipEventSynchronize(b) == hipSuccess) hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    return le == hipSuccess ? (double)ms : -2.0;
}

// Instructions of the measured kind each thread issues per call.
extern "C" uint64_t bwg_valu_ref_ops_per_thread(uint32_t iters) { return 16ull * kChains * iters; }
