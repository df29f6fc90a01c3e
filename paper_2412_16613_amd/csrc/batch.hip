// Batched execution of many ensembles (uneven networks, replica counts and
// plane widths) in one persistent launch.
//
// Work item = (ensemble, 64 consecutive words) for bit-sliced members, or
// (ensemble, 2 consecutive words) for members on the lanes engine (one
// replica per thread, same results); one wave takes one item at a time from
// a device queue ordered longest-first by the host, runs every pending event
// of its words (the same event loops as the per-ensemble kernels) and takes
// the next item until the queue is empty.
// Items never depend on each other: each word's events are its own, so the
// order in which waves take items changes nothing in the results.  Every
// wave leaves the loop once the queue counter passes the item count.

#include "wm_device.h"

namespace bwg {

// Plane buckets of the persistent kernel: (NB, BC) with run-time shift and
// unimolecular weight.  The host maps every network to the smallest bucket
// that holds it.
#define BWG_PERSIST_VARIANTS(X) \
    X(0, 6, 16)                 \
    X(1, 6, 20)                 \
    X(2, 6, 24)                 \
    X(3, 8, 20)                 \
    X(4, 8, 24)                 \
    X(5, 10, 24)                \
    X(6, 10, 28)                \
    X(7, 12, 24)                \
    X(8, 12, 28)                \
    X(9, 12, 32)                \
    X(10, 14, 32)

// The descriptor fields are the same for every lane of the wave; arguments
// of an out-of-line function are not known to be, so they are made
// wave-uniform (scalar registers, uniform branches on shifts and weights).
__device__ __forceinline__ uint32_t uni32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    return (uint64_t)uni32((uint32_t)v) | ((uint64_t)uni32((uint32_t)(v >> 32)) << 32);
}
template <typename T>
__device__ __forceinline__ T *uniptr(T *p)
{
    return (T *)uni64((uint64_t)p);
}
__device__ __forceinline__ WmArgs uniform_args(const WmArgs *ap, uint64_t max_events)
{
    WmArgs a = *ap;
    a.planes = uniptr(a.planes);
    a.E = uniptr(a.E);
    a.Etgt = uniptr(a.Etgt);
    a.real = uniptr(a.real);
    a.wp = uni64(a.wp);
    a.n_words = uni64(a.n_words);
    a.M = uni64(a.M);
    a.seed = uni64(a.seed);
    a.max_events = uni64(max_events);
    a.net_id = uni32(a.net_id);
    a.B = (int32_t)uni32((uint32_t)a.B);
    a.cu = uni32(a.cu);
    a.fa = (int32_t)uni32((uint32_t)a.fa);
    a.fi = (int32_t)uni32((uint32_t)a.fi);
    a.nb_mem = (int32_t)uni32((uint32_t)a.nb_mem);
    a.zs = 0;  // batches hold no shared-threshold members
    return a;
}

// One out-of-line function per bucket, so that each gets its own register
// allocation instead of the union of all of them.
template <int NB, int BC>
__device__ __noinline__ void wm_word_bucket(const WmArgs *ap, uint64_t w, uint64_t max_events)
{
    const WmArgs a = uniform_args(ap, max_events);
    wm_word<NB, BC, -1, -1>(a, w);
}

__device__ __noinline__ void wm_lanes_item(const WmArgs *ap, uint64_t w, uint32_t *sq,
                                           uint64_t max_events)
{
    const WmArgs a = uniform_args(ap, max_events);
    wm_lanes(a, w, sq);
}

#define BWG_PERSIST_CASE(id, nb, bc)        \
    case id:                                \
        wm_word_bucket<nb, bc>(&ens[bi.ens].a, w, max_events); \
        break;

__global__ __launch_bounds__(64, 2) void wm_persistent_kernel(const BatchEns *ens,
                                                              const BatchItem *items,
                                                              uint32_t n_items,
                                                              uint32_t *counter,
                                                              uint64_t max_events)
{
    // the lanes items' event rows (2 x kLanesHalfWords words), allocated at
    // launch only when the queue holds lanes items
    extern __shared__ __align__(16) uint32_t sq_dyn[];
    for (;;) {
        uint32_t it = 0;
        if (threadIdx.x == 0) it = atomicAdd(counter, 1u);
        it = __shfl(it, 0);
        if (it >= n_items) break;
        const BatchItem bi = items[it];
        if (bi.ens & BATCH_ITEM_LANES) {
            const int half = threadIdx.x >> 5;
            wm_lanes_item(&ens[bi.ens & ~BATCH_ITEM_LANES].a, (uint64_t)bi.word0 + half,
                          sq_dyn + half * kLanesHalfWords,
                          max_events);
            continue;
        }
        const int v = ens[bi.ens].variant;
        const uint64_t w = (uint64_t)bi.word0 + threadIdx.x;
        switch (v) {
            BWG_PERSIST_VARIANTS(BWG_PERSIST_CASE)
            default:
                break;
        }
    }
}

// Budgets of every ensemble of a batch in one launch: thread g belongs to
// the ensemble whose replica range [offset, offset + M) holds it.
__global__ void batch_budget_kernel(const BatchBudget *bb, int n_ens, uint64_t total, uint64_t g0)
{
    const uint64_t g = g0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int lo = 0, hi = n_ens - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (bb[mid].offset <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchBudget &b = bb[lo];
    const uint64_t i = g - b.offset;
    uint64_t K = 0;
    if (b.len) {
        const uint64_t adv = *b.adv;
        uint32_t o0, o1, o2, o3;
        philox4x32_10((uint32_t)adv, (DOM_BUDGET << 24) | ((uint32_t)(adv >> 32) & 0xFFFFu),
                      (uint32_t)i, b.net_id, (uint32_t)b.seed, (uint32_t)(b.seed >> 32), o0, o1,
                      o2, o3);
        const uint64_t u = (uint64_t)o0 | ((uint64_t)o1 << 32);
        uint64_t l = 0, h = b.len;
        while (l < h) {
            const uint64_t mid = (l + h) >> 1;
            if (b.T[mid] <= u)
                l = mid + 1;
            else
                h = mid;
        }
        K = (uint64_t)(b.k_lo + (int64_t)l);
    }
    b.Et[i] = b.E[i] + K;
}

// Queue reset and advance-index increments (a kernel, not a memset, so the
// sequence can be captured in a graph and replayed).
__global__ void batch_prologue_kernel(uint32_t *counter)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) counter[0] = 0;
}

__global__ void batch_epilogue_kernel(const BatchBudget *bb, int n_ens)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_ens) bb[k].adv[0] += 1;
}

hipError_t launch_persistent(const BatchEns *ens, const BatchItem *items, uint32_t n_items,
                             uint32_t *counter, int waves, uint64_t max_events, bool lanes,
                             hipStream_t s)
{
    const size_t lds = lanes ? 2 * kLanesHalfWords * sizeof(uint32_t) : 0;
    hipLaunchKernelGGL(wm_persistent_kernel, dim3((uint32_t)waves), dim3(64), lds, s, ens, items,
                       n_items, counter, max_events);
    return hipGetLastError();
}

hipError_t launch_batch_budget(const BatchBudget *bb, int n_ens, uint64_t total, hipStream_t s)
{
    return launch_pieces(total, 256, [&](uint64_t g0, dim3 g) {
        hipLaunchKernelGGL(batch_budget_kernel, g, dim3(256), 0, s, bb, n_ens, total, g0);
    });
}

hipError_t launch_batch_prologue(uint32_t *counter, hipStream_t s)
{
    hipLaunchKernelGGL(batch_prologue_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_batch_epilogue(const BatchBudget *bb, int n_ens, hipStream_t s)
{
    hipLaunchKernelGGL(batch_epilogue_kernel, dim3((uint32_t)((n_ens + 63) / 64)), dim3(64), 0,
                       s, bb, n_ens);
    return hipGetLastError();
}

#ifndef __HIP_DEVICE_COMPILE__
#define BWG_PERSIST_ENTRY(id, nb, bc) {id, nb, bc},
const PersistVariant kPersistVariants[] = {BWG_PERSIST_VARIANTS(BWG_PERSIST_ENTRY)};
const int kPersistVariantCount = sizeof(kPersistVariants) / sizeof(kPersistVariants[0]);
#endif

}  // namespace bwg
