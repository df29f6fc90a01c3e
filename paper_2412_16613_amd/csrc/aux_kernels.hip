// Initial states, event budgets, readouts and the ee histogram.

#include "bitops.h"
#include "bwg_internal.h"

namespace bwg {

// ---- initial states --------------------------------------------------------

// Every replica starts from the same counts: plane q of species x is all ones
// on live lanes where bit q of counts[x] is set.
__global__ void init_fixed_kernel(uint32_t *planes, int S, int nb, uint64_t wp, uint64_t M,
                                  SpeciesCounts c, uint64_t *E, uint64_t *Et, uint64_t *real)
{
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= wp) return;
    const uint64_t base = 32 * w;
    uint32_t live = 0;
    if (base < M) live = (M - base) >= 32 ? 0xFFFFFFFFu : ((1u << (M - base)) - 1u);
    for (int x = 0; x < S; ++x)
        for (int q = 0; q < nb; ++q)
            planes[((uint64_t)x * nb + q) * wp + w] = ((c.v[x] >> q) & 1) ? live : 0u;
    for (int l = 0; l < 32; ++l) {
        E[base + l] = 0;
        Et[base + l] = 0;
    }
    real[w] = 0;
}

// Multinomial start of the paper's experiment: each molecule is L, D or A
// with probability 1/4, 1/4, 1/2 from two random bits (00 -> L, 01 -> D,
// 1x -> A); molecule m uses bits 2(m mod 64), 2(m mod 64)+1 of the 128-bit
// INIT draw (chunk m/64, replica i).  One thread per replica; the counts are
// packed into planes with one wave ballot per plane.
__device__ __forceinline__ void multinomial_counts(uint64_t i, int64_t n_tot, uint64_t seed,
                                                   uint32_t net_id, int32_t &nL,
                                                   int32_t &nD, int32_t &nA)
{
    nL = nD = nA = 0;
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
}

__global__ void init_multinomial_kernel(uint32_t *planes, int nb, uint64_t wp, uint64_t M,
                                        int64_t n_tot, uint64_t seed, uint32_t net_id,
                                        uint64_t *E, uint64_t *Et, uint64_t *real, uint64_t i0)
{
    // blockDim is a multiple of 64 and the pieces cover 32*wp replicas exactly
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < M;
    int32_t c[3] = {0, 0, 0};
    if (ok) multinomial_counts(i, n_tot, seed, net_id, c[0], c[1], c[2]);
    const uint64_t w = i >> 5;
    const int lane = threadIdx.x & 63;
    for (int x = 0; x < 3; ++x)
        for (int q = 0; q < nb; ++q) {
            const uint64_t bits = __ballot(ok && ((c[x] >> q) & 1));
            if ((lane & 31) == 0)
                planes[((uint64_t)x * nb + q) * wp + w] =
                    lane ? (uint32_t)(bits >> 32) : (uint32_t)bits;
        }
    E[i] = 0;
    Et[i] = 0;
    if ((i & 31) == 0) real[w] = 0;
}

// ---- event budgets -----------------------------------------------------------

// Etgt[i] = E[i] + K_i with K_i = k_lo + #{j : T[j] <= u_i} (u_i the BUDGET
// draw of replica i for this advance) or the fixed count.
__device__ __forceinline__ uint64_t draw_budget(const uint64_t *T, uint64_t len, int64_t k_lo,
                                                uint64_t seed, uint32_t net_id, uint64_t adv,
                                                uint64_t i)
{
    uint32_t o0, o1, o2, o3;
    philox4x32_10((uint32_t)adv, (DOM_BUDGET << 24) | ((uint32_t)(adv >> 32) & 0xFFFFu),
                  (uint32_t)i, net_id, (uint32_t)seed, (uint32_t)(seed >> 32), o0, o1, o2, o3);
    const uint64_t u = (uint64_t)o0 | ((uint64_t)o1 << 32);
    uint64_t lo = 0, hi = len;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (T[mid] <= u)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (uint64_t)(k_lo + (int64_t)lo);
}

// The advance index is read from device memory so that a captured graph of
// an advance draws new budgets on every replay.
__global__ void budget_kernel(const uint64_t *T, uint64_t len, int64_t k_lo, uint64_t fixed_k,
                              int use_table, uint64_t seed, uint32_t net_id,
                              const uint64_t *adv_dev, uint64_t M, const uint64_t *E,
                              uint64_t *Et, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    uint64_t K = fixed_k;
    if (use_table) K = draw_budget(T, len, k_lo, seed, net_id, *adv_dev, i);
    Et[i] = E[i] + K;
}

__global__ void add_u64_kernel(uint64_t *p, uint64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] += v;
}

// ---- readouts ----------------------------------------------------------------

__device__ __forceinline__ int32_t plane_count(const uint32_t *planes, int x, int nb,
                                               uint64_t wp, uint64_t w, int lane)
{
    int32_t v = 0;
    for (int q = 0; q < nb; ++q)
        v |= (int32_t)((planes[((uint64_t)x * nb + q) * wp + w] >> lane) & 1u) << q;
    return v;
}

__global__ void read_counts_planes_kernel(const uint32_t *planes, int S, int nb, uint64_t wp,
                                          uint64_t M, int32_t *dst, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const uint64_t w = i >> 5;
    const int lane = (int)(i & 31);
    for (int x = 0; x < S; ++x) dst[S * i + x] = plane_count(planes, x, nb, wp, w, lane);
}

__global__ void read_counts_plain_kernel(const int32_t *counts, uint64_t M, int32_t *dst,
                                         uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * M) return;
    dst[i] = counts[i];
}

__global__ void fill_u64_kernel(uint64_t *dst, uint64_t n, uint64_t v, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

// bin = min(n_bins-1, floor((N_L - N_D + N_tot) n_bins / (2 N_tot))); block
// histogram in LDS, then one global atomic per non-empty bin.
__global__ void histogram_kernel(const uint32_t *planes, const int32_t *counts, int nb,
                                 uint64_t wp, uint64_t M, int64_t n_tot, int n_bins,
                                 uint64_t *dst, uint64_t i0)
{
    extern __shared__ uint32_t hist[];
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) {
        int32_t nl, nd;
        if (planes) {
            const uint64_t w = i >> 5;
            const int lane = (int)(i & 31);
            nl = plane_count(planes, 0, nb, wp, w, lane);
            nd = plane_count(planes, 1, nb, wp, w, lane);
        } else {
            nl = counts[3 * i];
            nd = counts[3 * i + 1];
        }
        int64_t b = ((int64_t)(nl - nd) + n_tot) * n_bins / (2 * n_tot);
        if (b > n_bins - 1) b = n_bins - 1;
        if (b < 0) b = 0;
        atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (hist[b]) atomicAdd((unsigned long long *)&dst[b], (unsigned long long)hist[b]);
}

// Counts of the selected replicas into dst[j * 3 + x]; an index at or past
// M gives -1 for every species.
__global__ void gather_counts_kernel(const uint32_t *planes, const int32_t *counts, int nb,
                                     uint64_t wp, uint64_t M, const uint32_t *sel, uint32_t n_sel,
                                     int32_t *dst, uint64_t i0)
{
    const uint64_t j = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_sel) return;
    const uint64_t i = sel[j];
    for (int x = 0; x < 3; ++x) {
        int32_t v = -1;
        if (i < M)
            v = planes ? plane_count(planes, x, nb, wp, i >> 5, (int)(i & 31)) : counts[3 * i + x];
        dst[3 * j + x] = v;
    }
}

// first[i] = k for every replica that has no entry yet (0xFFFFFFFF) and whose
// |N_L - N_D| has reached the threshold.
__global__ void first_passage_kernel(const uint32_t *planes, const int32_t *counts, int nb,
                                     uint64_t wp, uint64_t M, int32_t threshold, uint32_t k,
                                     uint32_t *first, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M || first[i] != 0xFFFFFFFFu) return;
    int32_t nl, nd;
    if (planes) {
        nl = plane_count(planes, 0, nb, wp, i >> 5, (int)(i & 31));
        nd = plane_count(planes, 1, nb, wp, i >> 5, (int)(i & 31));
    } else {
        nl = counts[3 * i];
        nd = counts[3 * i + 1];
    }
    const int32_t d = nl - nd;
    if ((d < 0 ? -d : d) >= threshold) first[i] = k;
}

__global__ void copy_u64_kernel(const uint64_t *src, uint64_t *dst, uint64_t n, uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// dst[slot] = sum(src[0..n)) with one block (used by stats, not hot).
__global__ void sum_u64_kernel(const uint64_t *src, uint64_t n, uint64_t *dst, int slot)
{
    __shared__ unsigned long long part[256];
    unsigned long long s = 0;
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) s += src[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[slot] = part[0];
}

// ---- launchers -----------------------------------------------------------------

static inline dim3 grid_for(uint64_t n, int block)
{
    return dim3((uint32_t)((n + block - 1) / block));
}

hipError_t launch_init_fixed(uint32_t *planes, int S, int nb, uint64_t wp, uint64_t M,
                             const int32_t *c, uint64_t *E, uint64_t *Et, uint64_t *real,
                             hipStream_t s)
{
    if (S < 1 || S > 8) return hipErrorInvalidValue;  // SpeciesCounts holds 8
    SpeciesCounts sc{};
    for (int x = 0; x < S; ++x) sc.v[x] = c[x];
    hipLaunchKernelGGL(init_fixed_kernel, grid_for(wp, 128), dim3(128), 0, s, planes, S, nb, wp,
                       M, sc, E, Et, real);
    return hipGetLastError();
}

hipError_t launch_init_multinomial(uint32_t *planes, int nb, uint64_t wp, uint64_t M,
                                   int64_t n_tot, uint64_t seed, uint32_t net_id, uint64_t *E,
                                   uint64_t *Et, uint64_t *real, hipStream_t s)
{
    // 32*wp is a multiple of 128 (wp is padded to 64 words)
    return launch_pieces(32 * wp, 128, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(init_multinomial_kernel, g, dim3(128), 0, s, planes, nb, wp, M, n_tot,
                           seed, net_id, E, Et, real, i0);
    });
}

hipError_t launch_budget(const uint64_t *T, uint64_t len, int64_t k_lo, uint64_t fixed_k,
                         int use_table, uint64_t seed, uint32_t net_id, const uint64_t *adv_dev,
                         uint64_t M, const uint64_t *E, uint64_t *Et, hipStream_t s)
{
    return launch_pieces(M, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(budget_kernel, g, dim3(256), 0, s, T, len, k_lo, fixed_k, use_table,
                           seed, net_id, adv_dev, M, E, Et, i0);
    });
}

hipError_t launch_add_u64(uint64_t *p, uint64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(add_u64_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s)
{
    return launch_pieces(n, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(fill_u64_kernel, g, dim3(256), 0, s, p, n, v, i0);
    });
}

hipError_t launch_read_counts_planes(const uint32_t *planes, int S, int nb, uint64_t wp,
                                     uint64_t M, int32_t *dst, hipStream_t s)
{
    return launch_pieces(M, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(read_counts_planes_kernel, g, dim3(256), 0, s, planes, S, nb, wp, M,
                           dst, i0);
    });
}

hipError_t launch_read_counts_plain(const int32_t *counts, uint64_t M, int32_t *dst,
                                    hipStream_t s)
{
    return launch_pieces(3 * M, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(read_counts_plain_kernel, g, dim3(256), 0, s, counts, M, dst, i0);
    });
}

hipError_t launch_histogram(const uint32_t *planes, const int32_t *counts, int nb, uint64_t wp,
                            uint64_t M, int64_t n_tot, int n_bins, uint64_t *dst,
                            hipStream_t s)
{
    const hipError_t e = launch_fill_u64(dst, (uint64_t)n_bins, 0ull, s);
    if (e != hipSuccess) return e;
    return launch_pieces(M, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(histogram_kernel, g, dim3(256), (size_t)n_bins * sizeof(uint32_t), s,
                           planes, counts, nb, wp, M, n_tot, n_bins, dst, i0);
    });
}

hipError_t launch_gather_counts(const uint32_t *planes, const int32_t *counts, int nb,
                                uint64_t wp, uint64_t M, const uint32_t *sel, uint32_t n_sel,
                                int32_t *dst, hipStream_t s)
{
    return launch_pieces(n_sel, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(gather_counts_kernel, g, dim3(256), 0, s, planes, counts, nb, wp, M,
                           sel, n_sel, dst, i0);
    });
}

hipError_t launch_first_passage(const uint32_t *planes, const int32_t *counts, int nb,
                                uint64_t wp, uint64_t M, int32_t threshold, uint32_t k,
                                uint32_t *first, hipStream_t s)
{
    return launch_pieces(M, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(first_passage_kernel, g, dim3(256), 0, s, planes, counts, nb, wp, M,
                           threshold, k, first, i0);
    });
}

hipError_t launch_copy_u64(const uint64_t *src, uint64_t *dst, uint64_t n, hipStream_t s)
{
    return launch_pieces(n, 256, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(copy_u64_kernel, g, dim3(256), 0, s, src, dst, n, i0);
    });
}

hipError_t launch_sum_u64(const uint64_t *src, uint64_t n, uint64_t *dst, int slot,
                          hipStream_t s)
{
    hipLaunchKernelGGL(sum_u64_kernel, dim3(1), dim3(256), 0, s, src, n, dst, slot);
    return hipGetLastError();
}

}  // namespace bwg
