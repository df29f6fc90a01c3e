// Compartment (lattice) kernels: initial site states, the component schedule
// of each 2048-replica group, the layered event kernel and the readouts.
//
// The paper presents the bitwise method for one well-mixed reactor and names
// ensembles of small compartments as what it is meant for (Sec. 1, Sec. 6).
// Here every replica is a periodic lx x ly lattice of Frank reactors (site
// counts L, D, A in P bit planes each, site total at most T = 2^P - 1) whose
// molecules hop to the 4 neighbours.  The uniformised chain draws, per event,
// one component shared by the replicas of a group -- the reaction of a site,
// or a hop out of a site in one direction -- and per replica a threshold
// (reaction: B_r planes, first crossing of the site's cumulative weights, the
// Sec. 4 comparator) or a hop index j in [0, T] (A if j < n_A, L if
// j < n_A + n_L, D if j < n_site; blocked when the destination is full).
//
// Events of one group that touch disjoint sites commute, so the schedule
// kernel sorts each chunk of the group's component sequence into greedy
// layers of pairwise disjoint events; the event kernel runs one layer at a
// time, every event of a layer in its own thread, on the planes of one word
// (32 replicas).  Each replica still applies exactly its own events, in an
// order that only permutes commuting events.

#include "bitops.h"
#include "bwg.h"
#include "bwg_internal.h"

namespace bwg {

// ---- draws -------------------------------------------------------------------

// Component of event e of a group: uniform in [0, C) from 64-bit COMPONENT
// draws by Lemire's multiply-and-reject (thresh = 2^64 mod C); the attempt
// index is part of the counter, and the 256th attempt is taken as it is.
__device__ __forceinline__ uint64_t lat_component(uint64_t seed, uint32_t net_id, uint32_t group,
                                                  uint64_t e, uint64_t C, uint64_t thresh)
{
    uint64_t u = 0;
    for (uint32_t attempt = 0; attempt < 256; ++attempt) {
        uint32_t o0, o1, o2, o3;
        philox4x32_10((uint32_t)e,
                      (DOM_COMPONENT << 24) | (attempt << 16) | ((uint32_t)(e >> 32) & 0xFFFFu),
                      group, net_id, (uint32_t)seed, (uint32_t)(seed >> 32), o0, o1, o2, o3);
        u = (uint64_t)o0 | ((uint64_t)o1 << 32);
        if (u * C >= thresh) break;
    }
    return __umul64hi(u, C);
}

// A uniform in {lo..hi} for (replica i, site s): 32-bit Lemire with rejection
// over the four outputs of successive INIT draws.
__device__ __forceinline__ int32_t lat_init_count(uint64_t seed, uint32_t net_id, uint64_t i,
                                                  uint32_t s, int32_t lo, int32_t hi)
{
    const uint32_t R = (uint32_t)(hi - lo + 1);
    const uint32_t thresh = (0u - R) % R;
    for (uint32_t attempt = 0; attempt < 65536; ++attempt) {
        uint32_t o[4];
        philox4x32_10(s, (DOM_INIT << 24) | (1u << 23) | attempt, (uint32_t)i, net_id,
                      (uint32_t)seed, (uint32_t)(seed >> 32), o[0], o[1], o[2], o[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t m = (uint64_t)o[k] * R;
            if ((uint32_t)m >= thresh) return lo + (int32_t)(m >> 32);
        }
    }
    return lo;
}

__device__ __forceinline__ uint32_t lat_neighbour(const LatShape &sh, uint32_t s, uint32_t dir)
{
    uint32_t x = s % (uint32_t)sh.lx, y = s / (uint32_t)sh.lx;
    if (dir == 0)
        x = x + 1 == (uint32_t)sh.lx ? 0 : x + 1;
    else if (dir == 1)
        x = x == 0 ? sh.lx - 1 : x - 1;
    else if (dir == 2)
        y = y + 1 == (uint32_t)sh.ly ? 0 : y + 1;
    else
        y = y == 0 ? sh.ly - 1 : y - 1;
    return y * (uint32_t)sh.lx + x;
}

// ---- layout ----------------------------------------------------------------
// Site planes of word w in group g = w / 64: a group stores, site by site, the
// 3P planes of each of its 64 words (padded), so the planes of one site of
// consecutive words are contiguous:
//   planes[((g S + s) 64 + (w mod 64)) 3P + x P + q],  species x in (L, D, A).
__device__ __forceinline__ uint32_t *site_planes(uint32_t *planes, uint64_t w, uint32_t s,
                                                 int S, int NP)
{
    return planes + (((w >> 6) * (uint64_t)S + s) * 64 + (w & 63)) * (uint64_t)NP;
}
__device__ __forceinline__ const uint32_t *site_planes(const uint32_t *planes, uint64_t w,
                                                       uint32_t s, int S, int NP)
{
    return planes + (((w >> 6) * (uint64_t)S + s) * 64 + (w & 63)) * (uint64_t)NP;
}

// ---- initial states -------------------------------------------------------------

// mode 0: every site of every replica holds site[s] (sites = null: site0 for
// all sites); one thread per (word, site).
__global__ void lat_init_fixed_kernel(uint32_t *planes, uint64_t words, uint64_t M, int S, int P,
                                      const int32_t *sites, int32_t l0, int32_t d0, int32_t a0,
                                      uint64_t *E, uint64_t *Et, uint64_t *real, uint64_t *blocked)
{
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t s = blockIdx.y;
    if (w >= words) return;
    const uint64_t rem = M - 32 * w;
    const uint32_t live = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    int32_t c[3] = {l0, d0, a0};
    if (sites) {
        c[0] = sites[3 * s];
        c[1] = sites[3 * s + 1];
        c[2] = sites[3 * s + 2];
    }
    uint32_t *p = site_planes(planes, w, s, S, 3 * P);
    for (int x = 0; x < 3; ++x)
        for (int q = 0; q < P; ++q) p[x * P + q] = ((c[x] >> q) & 1) ? live : 0u;
    if (s == 0) {
        for (int l = 0; l < 32; ++l) {
            E[32 * w + l] = 0;
            Et[32 * w + l] = 0;
        }
        real[w] = 0;
        blocked[w] = 0;
    }
}

// mode 1: A uniform in {lo..hi} per (replica, site), L = D = 0.  A wave holds
// 64 replicas (two words) of one site and packs their counts with ballots.
__global__ void lat_init_uniform_kernel(uint32_t *planes, uint64_t words, uint64_t M, int S, int P,
                                       int32_t lo, int32_t hi, uint64_t seed, uint32_t net_id,
                                       uint64_t *E, uint64_t *Et, uint64_t *real,
                                       uint64_t *blocked)
{
    // blockDim.x is a multiple of 64; grid.x covers 64 * ceil(words / 2) replicas
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t s = blockIdx.y;
    const bool ok = i < M;
    const int32_t a = ok ? lat_init_count(seed, net_id, i, s, lo, hi) : 0;
    const uint64_t w = i >> 5;
    const int lane = threadIdx.x & 63;
    for (int q = 0; q < P; ++q) {
        const uint64_t bits = __ballot(ok && ((a >> q) & 1));
        if ((lane & 31) == 0 && w < words) {
            uint32_t *p = site_planes(planes, w, s, S, 3 * P);
            p[q] = 0u;
            p[P + q] = 0u;
            p[2 * P + q] = lane ? (uint32_t)(bits >> 32) : (uint32_t)bits;
        }
    }
    if (s == 0 && w < words) {
        E[i] = 0;
        Et[i] = 0;
        if ((i & 31) == 0) {
            real[w] = 0;
            blocked[w] = 0;
        }
    }
}

// ---- schedule -------------------------------------------------------------------
// One wave per (group, chunk of LAT_CH events).  Slot layout (uint32):
//   recs[LAT_CH]   events in layer order: (offset in chunk) << 16 | site << 3 | kind
//   tmp[LAT_CH]    per event: layer << 16 | site << 3 | kind (layer 0: outside)
//   offs[0]        number of layers; offs[1 + L] = first event of layer L
//                  (L = 0 .. layers), so layer L is recs[offs[1+L] .. offs[2+L]).
// kind 0 is the site's reaction component, 1 + d a hop in direction d.

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int o = 32; o; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    for (int o = 32; o; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    for (int o = 32; o; o >>= 1) {
        const uint32_t lo = __shfl_xor((int)(uint32_t)v, o, 64);
        const uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), o, 64);
        v = min(v, (uint64_t)lo | ((uint64_t)hi << 32));
    }
    return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    for (int o = 32; o; o >>= 1) {
        const uint32_t lo = __shfl_xor((int)(uint32_t)v, o, 64);
        const uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), o, 64);
        v = max(v, (uint64_t)lo | ((uint64_t)hi << 32));
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up((int)v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__global__ __launch_bounds__(64) void lat_schedule_kernel(LatArgs a)
{
    __shared__ uint16_t last[LAT_MAX_SITES];
    __shared__ uint32_t first[LAT_MAX_SITES];
    __shared__ uint32_t hist[LAT_CH];  // two 16-bit counters per word, key = 2 layer + hop

    const int lane = threadIdx.x;
    const uint32_t ci = blockIdx.x % a.n_chunks;
    const uint32_t g = blockIdx.x / a.n_chunks;
    uint32_t *slot = a.sched + ((uint64_t)g * LAT_NCB + ci) * LAT_SLOT;
    uint32_t *recs = slot, *tmp = slot + LAT_CH, *offs = slot + 2 * LAT_CH;
    const LatShape &sh = a.sh;

    // events of this chunk that some pending replica of the group runs
    const uint64_t r0 = (uint64_t)g * LAT_GROUP_WORDS * 32;
    const uint64_t r1 = min(a.M, r0 + LAT_GROUP_WORDS * 32);
    uint64_t lo = ~0ull, hi = 0;
    for (uint64_t i = r0 + lane; i < r1; i += 64) {
        const uint64_t e0 = a.E[i], e1 = a.Et[i];
        if (e0 < e1) {
            lo = min(lo, e0);
            hi = max(hi, e1);
        }
    }
    lo = wave_min_u64(lo);
    hi = wave_max_u64(hi);
    const uint64_t cbase = a.base + (uint64_t)(a.chunk0 + ci) * LAT_CH;
    const uint64_t clo = max(cbase, lo), chi = min(cbase + LAT_CH, hi);
    if (clo >= chi) {
        if (lane == 0) offs[0] = 0;
        return;
    }
    for (int k = lane; k < sh.S; k += 64) {
        last[k] = 0;
        first[k] = ~0u;
    }
    for (int k = lane; k < LAT_CH; k += 64) hist[k] = 0;
    __syncthreads();

    // greedy layers: an event's layer is one more than the last layer that
    // touched either of its sites; within a batch of 64 events, a lane is
    // settled in the round where it is the earliest unsettled lane at both
    // of its sites, so settled lanes of one round touch disjoint sites.
    uint32_t maxlay = 0;
    for (uint32_t b = 0; b < LAT_CH; b += 64) {
        const uint32_t off = b + lane;
        const uint64_t e = cbase + off;
        const bool in = e >= clo && e < chi;
        uint32_t s = 0, s2 = 0, kind = 0;
        if (in) {
            const uint64_t comp = lat_component(a.seed, a.net_id, g, e, sh.C, sh.thresh);
            const uint64_t q = comp / sh.Wsite;
            const uint64_t r = comp - q * sh.Wsite;
            s = (uint32_t)q;
            kind = r < sh.W_R ? 0u : 1u + (uint32_t)((r - sh.W_R) / sh.W_H);
            s2 = kind ? lat_neighbour(sh, s, kind - 1) : s;
        }
        bool pend = in;
        uint32_t lay = 0;
        while (__any(pend)) {
            if (pend) {
                atomicMin(&first[s], (uint32_t)lane);
                atomicMin(&first[s2], (uint32_t)lane);
            }
            __syncthreads();
            bool settled = false;
            if (pend) settled = first[s] == (uint32_t)lane && first[s2] == (uint32_t)lane;
            if (settled) {
                lay = 1u + max((uint32_t)last[s], (uint32_t)last[s2]);
                last[s] = (uint16_t)lay;
                last[s2] = (uint16_t)lay;
            }
            __syncthreads();
            if (pend) {
                first[s] = ~0u;
                first[s2] = ~0u;
            }
            __syncthreads();
            pend = pend && !settled;
        }
        if (in) {
            const uint32_t key = 2 * (lay - 1) + (kind != 0);
            atomicAdd(&hist[key >> 1], 1u << (16 * (key & 1)));
            maxlay = max(maxlay, lay);
            tmp[off] = (lay << 16) | (s << 3) | kind;
        } else {
            tmp[off] = 0;
        }
    }
    const uint32_t nl = wave_max_u32(maxlay);
    __syncthreads();

    // exclusive prefix over keys 0 .. 2 nl - 1, written back as cursors
    uint32_t run = 0;
    for (uint32_t kb = 0; kb < 2 * nl; kb += 64) {
        const uint32_t k = kb + lane;
        const uint32_t cnt = k < 2 * nl ? (hist[k >> 1] >> (16 * (k & 1))) & 0xFFFFu : 0u;
        const uint32_t incl = wave_incl_scan(cnt, lane);
        const uint32_t excl = run + incl - cnt;
        const uint32_t odd = __shfl_down((int)excl, 1, 64);
        __syncthreads();
        if (k < 2 * nl && (k & 1) == 0) {
            hist[k >> 1] = excl | (odd << 16);
            offs[1 + (k >> 1)] = excl;
        }
        run += __shfl((int)incl, 63, 64);
        __syncthreads();
    }
    if (lane == 0) {
        offs[0] = nl;
        offs[1 + nl] = run;
    }
    __syncthreads();
    for (uint32_t b = 0; b < LAT_CH; b += 64) {
        const uint32_t off = b + lane;
        const uint32_t t = tmp[off];
        const uint32_t lay = t >> 16;
        if (lay) {
            const uint32_t key = 2 * (lay - 1) + ((t & 7u) != 0);
            const uint32_t sh16 = 16 * (key & 1);
            const uint32_t old = atomicAdd(&hist[key >> 1], 1u << sh16);
            recs[(old >> sh16) & 0xFFFFu] = (off << 16) | (t & 0xFFFFu);
        }
    }
}

// ---- event kernel ------------------------------------------------------------

// acc (BC planes) += p << SH over planes [SH, BC).
template <int BC, int WP, int SH>
__device__ __forceinline__ void add_shifted(uint32_t (&acc)[BC], const uint32_t (&p)[WP])
{
    uint32_t cy = 0;
#pragma unroll
    for (int q = SH; q < BC; ++q) {
        const uint32_t v = (q - SH < WP) ? p[q - SH] : 0u;
        const uint32_t s = BWG_OP3(acc[q], v, cy, L_XOR3);
        if (q + 1 < BC) cy = BWG_OP3(acc[q], v, cy, L_MAJ);
        acc[q] = s;
    }
}

// Run-time shift: one compile-time addition is taken (wave-uniform branch).
template <int BC, int WP, int SH = 0>
__device__ __forceinline__ void add_dispatch(int sh, uint32_t (&acc)[BC], const uint32_t (&p)[WP])
{
    if constexpr (SH < BC) {
        if (sh == SH) {
            add_shifted<BC, WP, SH>(acc, p);
            return;
        }
        add_dispatch<BC, WP, SH + 1>(sh, acc, p);
    }
}

template <int BC, int WP, int64_t K, int k = 0>
__device__ __forceinline__ void add_bits(uint32_t (&acc)[BC], const uint32_t (&p)[WP])
{
    if constexpr (k < BC) {
        if constexpr ((K >> k) & 1) add_shifted<BC, WP, k>(acc, p);
        add_bits<BC, WP, K, k + 1>(acc, p);
    }
}

// acc += c * p: K >= 0 is the constant at compile time, else c at run time
// (one shifted addition per set bit).
template <int BC, int WP, int64_t K>
__device__ __forceinline__ void add_const_mul(uint32_t (&acc)[BC], const uint32_t (&p)[WP],
                                              uint64_t c)
{
    if constexpr (K >= 0) {
        add_bits<BC, WP, K>(acc, p);
    } else {
        for (uint64_t cc = c; cc; cc &= cc - 1) add_dispatch<BC, WP>(__builtin_ctzll(cc), acc, p);
    }
}

// [n < S] per lane over BC planes.
template <int BC>
__device__ __forceinline__ uint32_t less_than(const uint32_t (&n)[BC], const uint32_t (&S)[BC])
{
    uint32_t br = 0;
#pragma unroll
    for (int q = 0; q < BC; ++q) br = BWG_OP3(n[q], S[q], br, L_BORROW);
    return br;
}

template <int W>
__device__ __forceinline__ uint32_t less_than_w(const uint32_t (&j)[W], const uint32_t (&x)[W])
{
    uint32_t br = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) br = BWG_OP3(j[q], x[q], br, L_BORROW);
    return br;
}

template <int W>
__device__ __forceinline__ void add_w(uint32_t (&out)[W], const uint32_t (&x)[W],
                                      const uint32_t (&y)[W])
{
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const uint32_t s = BWG_OP3(x[q], y[q], c, L_XOR3);
        c = BWG_OP3(x[q], y[q], c, L_MAJ);
        out[q] = s;
    }
}

template <int P>
__device__ __forceinline__ void load_site(const uint32_t *p, uint32_t (&l)[P], uint32_t (&d)[P],
                                          uint32_t (&a)[P])
{
    if constexpr (P == 4) {
        const uint4 *v = reinterpret_cast<const uint4 *>(p);
        const uint4 x = v[0], y = v[1], z = v[2];
        l[0] = x.x; l[1] = x.y; l[2] = x.z; l[3] = x.w;
        d[0] = y.x; d[1] = y.y; d[2] = y.z; d[3] = y.w;
        a[0] = z.x; a[1] = z.y; a[2] = z.z; a[3] = z.w;
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            l[q] = p[q];
            d[q] = p[P + q];
            a[q] = p[2 * P + q];
        }
    }
}

template <int P>
__device__ __forceinline__ void store_site(uint32_t *p, const uint32_t (&l)[P],
                                           const uint32_t (&d)[P], const uint32_t (&a)[P])
{
    if constexpr (P == 4) {
        uint4 *v = reinterpret_cast<uint4 *>(p);
        v[0] = make_uint4(l[0], l[1], l[2], l[3]);
        v[1] = make_uint4(d[0], d[1], d[2], d[3]);
        v[2] = make_uint4(a[0], a[1], a[2], a[3]);
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            p[q] = l[q];
            p[P + q] = d[q];
            p[2 * P + q] = a[q];
        }
    }
}

// Threshold planes 0 .. nq-1 of event e for the 32 lanes of word G (the
// EVENT draws of the well-mixed kernel); planes >= nq are zero.
template <int BC>
__device__ __forceinline__ void event_planes(uint32_t (&n)[BC], uint64_t seed, uint32_t net_id,
                                             uint32_t G, uint64_t e, int nq)
{
#pragma unroll
    for (int k = 0; 4 * k < BC; ++k) {
        uint32_t o[4] = {0, 0, 0, 0};
        if (4 * k < nq)
            philox4x32_10((uint32_t)e,
                          (DOM_EVENT << 24) | ((uint32_t)k << 16) | ((uint32_t)(e >> 32) & 0xFFFFu),
                          G, net_id, (uint32_t)seed, (uint32_t)(seed >> 32), o[0], o[1], o[2],
                          o[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (4 * k + j < BC) n[4 * k + j] = (4 * k + j < nq) ? o[j] : 0u;
    }
}

// Reaction component of a site (planes l, d, x already loaded, updated in
// place) for the lanes in act; returns the lanes whose state changed (the
// caller stores the planes if any did).
template <int P, int BC, int64_t CU, int64_t CA, int64_t CI>
__device__ __forceinline__ uint32_t lat_reaction(uint32_t (&l)[P], uint32_t (&d)[P],
                                                 uint32_t (&x)[P], const LatArgs &a, uint32_t G,
                                                 uint64_t e, uint32_t act)
{
    constexpr int WP = 2 * P;
    const LatShape &sh = a.sh;
    uint32_t n[BC];
    event_planes<BC>(n, a.seed, a.net_id, G, e, sh.B_r);

    // S_1 = cu A, S_2 = 2 cu A, S_3 = S_2 + c_a A L, S_4 = S_3 + c_a A D,
    // S_5 = S_4 + c_i L D (table order A->L, A->D, A+L->2L, A+D->2D, L+D->2A)
    uint32_t X[BC];
#pragma unroll
    for (int q = 0; q < BC; ++q) X[q] = 0;
    add_const_mul<BC, P, CU>(X, x, sh.cu);
    const uint32_t lt1 = less_than<BC>(n, X);
    uint32_t S[BC];
    S[0] = 0;
#pragma unroll
    for (int q = 1; q < BC; ++q) S[q] = X[q - 1];
    const uint32_t lt2 = less_than<BC>(n, S);
    uint32_t pr[WP];
    mul_planes<P, WP>(pr, x, l);
    add_const_mul<BC, WP, CA>(S, pr, sh.ca);
    const uint32_t lt3 = less_than<BC>(n, S);
    mul_planes<P, WP>(pr, x, d);
    add_const_mul<BC, WP, CA>(S, pr, sh.ca);
    const uint32_t lt4 = less_than<BC>(n, S);
    mul_planes<P, WP>(pr, l, d);
    add_const_mul<BC, WP, CI>(S, pr, sh.ci);
    const uint32_t lt5 = less_than<BC>(n, S);

    const uint32_t mL = (lt1 | (lt3 & ~lt2)) & act;
    const uint32_t mD = ((lt2 & ~lt1) | (lt4 & ~lt3)) & act;
    const uint32_t mI = lt5 & ~lt4 & act;
    const uint32_t ch = mL | mD | mI;
    if (ch) {
        add_pm1<P>(l, mL, mI);
        add_pm1<P>(d, mD, mI);
        add_m1_p2<P>(x, mL | mD, mI);
    }
    return ch;
}

// Hop component out of one site into another (planes already loaded,
// updated in place; self: the lattice is one site wide along that axis and
// the hop changes nothing).  Sets the lanes that moved (the caller stores
// both sites' planes if any did) and the lanes blocked by a full
// destination.
template <int P>
__device__ __forceinline__ void lat_hop(bool self, uint32_t (&l)[P],
                                        uint32_t (&d)[P], uint32_t (&x)[P], uint32_t (&l2)[P],
                                        uint32_t (&d2)[P], uint32_t (&x2)[P], const LatArgs &a,
                                        uint32_t G, uint64_t e, uint32_t act, uint32_t &moved,
                                        uint32_t &blocked)
{
    static_assert(P <= 4, "hop index from one Philox quad");
    uint32_t o[4];
    philox4x32_10((uint32_t)e, (DOM_EVENT << 24) | ((uint32_t)(e >> 32) & 0xFFFFu), G, a.net_id,
                  (uint32_t)a.seed, (uint32_t)(a.seed >> 32), o[0], o[1], o[2], o[3]);
    uint32_t j[P];
#pragma unroll
    for (int q = 0; q < P; ++q) j[q] = o[q];
    uint32_t al[P], tot[P];
    add_w<P>(al, x, l);     // site totals are at most T = 2^P - 1: no carry out
    add_w<P>(tot, al, d);
    const uint32_t hA = less_than_w<P>(j, x);
    const uint32_t cAL = less_than_w<P>(j, al);
    const uint32_t any = less_than_w<P>(j, tot) & act;
    const uint32_t sA = hA & act, sL = cAL & ~hA & act, sD = any & ~cAL;
    uint32_t t2[P], full = ~0u;
    add_w<P>(t2, x2, l2);
    add_w<P>(t2, t2, d2);
#pragma unroll
    for (int q = 0; q < P; ++q) full &= t2[q];
    const uint32_t mv = any & ~full;
    blocked = any & full;
    moved = self ? 0u : mv;
    if (self || !mv) return;
    add_pm1<P>(x, 0u, sA & mv);
    add_pm1<P>(l, 0u, sL & mv);
    add_pm1<P>(d, 0u, sD & mv);
    add_pm1<P>(x2, sA & mv, 0u);
    add_pm1<P>(l2, sL & mv, 0u);
    add_pm1<P>(d2, sD & mv, 0u);
}

// Lanes of a word that run event e (E_l <= e < Et_l); kept out of line so the
// 64 window bounds are not held in registers across the event loop.
__device__ __noinline__ uint32_t lanes_at(const uint64_t *sE, const uint64_t *sEt, uint32_t pend,
                                          uint64_t e)
{
    uint32_t act = 0;
    for (int l = 0; l < 32; ++l)
        if (((pend >> l) & 1u) && sE[l] <= e && e < sEt[l]) act |= 1u << l;
    return act;
}

// One workgroup per slice of WS consecutive words of a group, BLOCK
// threads: thread t works on word t mod WS of the slice and on every
// (BLOCK / WS)-th event of a layer, so the WS words of one event read
// WS * 12 contiguous planes.  A launch covers the band of groups
// [a.g0, a.g0 + a.ng): the host sizes bands so that their site planes fit the
// last-level (infinity) cache.  Slices are spread so that the slices of a
// group run on one XCD (workgroups go to the 8 XCDs in turn), where they
// share the group's schedule in L2.  Runs the events of chunks chunk0 ..
// chunk0+n_chunks-1 layer by layer.
//
// ST > 0 (P = 4): the planes of sites 0 .. ST/WS - 1 of the slice's words
// are copied into LDS when the launch starts and back when it ends, and
// every event on those sites reads and writes LDS instead of memory.  LDS
// holds ST = 3360 (site, word) pairs (158 KB of the CU's 160 KB): with 4-word
// slices the first 840 sites of each word, a fifth of a 64 x 64 lattice.
// Within a layer no two events share a site, so the LDS copy needs no more
// ordering than the memory planes do.  (One word per workgroup would hold
// 3392 sites, 83 % of a 64 x 64 lattice, but a word's layers hold ~550
// independent events on average, half of the 1024 threads a CU needs to
// hide latency: measured slower.)
template <int P, int BC, int64_t CU, int64_t CA, int64_t CI, int WS, int BLOCK, int ST>
__global__ __launch_bounds__(BLOCK, 1) void lat_event_kernel(LatArgs a)
{
    static_assert(ST == 0 || P == 4, "staging holds 12 planes per site and word");
    constexpr int NP = 3 * P;
    constexpr int NSL = LAT_GROUP_WORDS / WS;   // slices per group
    constexpr int EV = BLOCK / WS;              // events in flight per workgroup
    const uint32_t nwg = a.ng * NSL;
    const uint32_t per_xcd = (nwg + 7) / 8;
    const uint32_t v = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (v >= nwg) return;
    const uint32_t g = a.g0 + v / NSL;
    const uint64_t w0 = (uint64_t)g * LAT_GROUP_WORDS + (v % NSL) * WS;
    const uint64_t words = (a.M + 31) / 32;
    if (w0 >= words) return;
    const uint32_t tid = threadIdx.x, lw = tid % WS, slot = tid / WS;
    const uint64_t w = w0 + lw;
    __shared__ uint64_t sE[WS][32], sEt[WS][32];
    __shared__ uint32_t sred[2][WS];

    for (uint32_t i = tid; i < WS * 32; i += BLOCK) {
        const uint64_t r = 32 * w0 + i;
        const bool ok = r < a.M;
        sE[i / 32][i % 32] = ok ? a.E[r] : 0;
        sEt[i / 32][i % 32] = ok ? a.Et[r] : 0;
    }
    if (tid < 2 * WS) sred[tid / WS][tid % WS] = 0;
    __syncthreads();
    // window of this thread's word over its pending lanes (E < Et): [lo, hi)
    // holds every event of the word, [blo, bhi) the events every pending
    // lane runs; [wlo, whi) the union over the slice
    uint64_t lo = ~0ull, hi = 0, blo = 0, bhi = ~0ull, wlo = ~0ull, whi = 0;
    uint32_t pend = 0;
    for (int l = 0; l < 32; ++l) {
        const uint64_t e0 = sE[lw][l], e1 = sEt[lw][l];
        if (e0 < e1) {
            pend |= 1u << l;
            lo = min(lo, e0);
            hi = max(hi, e1);
            blo = max(blo, e0);
            bhi = min(bhi, e1);
        }
    }
    for (int k = 0; k < WS * 32; ++k) {
        const uint64_t e0 = sE[k / 32][k % 32], e1 = sEt[k / 32][k % 32];
        if (e0 < e1) {
            wlo = min(wlo, e0);
            whi = max(whi, e1);
        }
    }
    const int S = a.sh.S;
    uint32_t n_real = 0, n_blocked = 0;
    // the launch's events of this slice: [wlo, whi) within its chunks
    const uint64_t c_lo = a.base + (uint64_t)a.chunk0 * LAT_CH;
    const uint64_t c_hi = c_lo + (uint64_t)a.n_chunks * LAT_CH;
    const bool runs = whi > wlo && wlo < c_hi && whi > c_lo;
    // stage[(st WS + word) 3 + part]: the slice's WS words of site st
    __shared__ uint4 stage[ST > 0 ? 3 * ST : 1];
    const uint32_t nst = ST > 0 ? min((uint32_t)S, (uint32_t)(ST / WS)) : 0u;
    if (ST > 0 && runs) {
        for (uint32_t k = tid; k < 3 * WS * nst; k += BLOCK)
            stage[k] = reinterpret_cast<const uint4 *>(
                site_planes(a.planes, w0 + (k / 3) % WS, k / (3 * WS), S, NP))[k % 3];
        __syncthreads();
    }
    // planes of site st of this thread's word: LDS for staged sites.  The two
    // cases stay separate instructions (LDS and memory loads wait on their own
    // counters, so the next event's memory loads still overlap this event)
    auto load_at = [&](uint32_t st, uint32_t (&l_)[P], uint32_t (&d_)[P], uint32_t (&x_)[P]) {
        if (ST > 0 && st < nst)
            load_site<P>(reinterpret_cast<const uint32_t *>(&stage[3 * (st * WS + lw)]), l_, d_, x_);
        else
            load_site<P>(site_planes(a.planes, w, st, S, NP), l_, d_, x_);
    };
    auto store_at = [&](uint32_t st, const uint32_t (&l_)[P], const uint32_t (&d_)[P],
                        const uint32_t (&x_)[P]) {
        if (ST > 0 && st < nst)
            store_site<P>(reinterpret_cast<uint32_t *>(&stage[3 * (st * WS + lw)]), l_, d_, x_);
        else
            store_site<P>(site_planes(a.planes, w, st, S, NP), l_, d_, x_);
    };
    if (runs) {
        for (uint32_t c = 0; c < a.n_chunks; ++c) {
            const uint32_t *slotp = a.sched + ((uint64_t)g * LAT_NCB + c) * LAT_SLOT;
            const uint32_t *recs = slotp;
            const uint32_t *offs = slotp + 2 * LAT_CH;
            const uint64_t cbase = a.base + (uint64_t)(a.chunk0 + c) * LAT_CH;
            if (cbase >= whi || cbase + LAT_CH <= wlo) continue;
            const uint32_t nl = offs[0];
            for (uint32_t L = 0; L < nl; ++L) {
                const uint32_t end = offs[2 + L];
                // the planes of this thread's next event of the layer are
                // loaded while the current one computes: events of a layer
                // touch disjoint sites, so nothing else writes them meanwhile
                uint32_t idx = offs[1 + L] + slot;
                uint64_t e = 0;
                uint32_t s = 0, s2 = 0, kind = 0, act = 0;
                uint32_t l[P], d[P], x[P], l2[P], d2[P], x2[P];
                auto fetch = [&](uint32_t i) {
                    const uint32_t rec = recs[i];
                    e = cbase + (rec >> 16);
                    act = 0;
                    if (e >= lo && e < hi)
                        act = (e >= blo && e < bhi) ? pend : lanes_at(sE[lw], sEt[lw], pend, e);
                    s = (rec >> 3) & 0x1FFFu;
                    kind = rec & 7u;
                    s2 = kind ? lat_neighbour(a.sh, s, kind - 1) : s;
                    if (act) {
                        load_at(s, l, d, x);
                        if (s2 != s) load_at(s2, l2, d2, x2);
                    }
                };
                if (idx < end) fetch(idx);
                while (idx < end) {
                    const uint64_t e_c = e;
                    const uint32_t s_c = s, s2_c = s2, kind_c = kind, act_c = act;
                    uint32_t lc[P], dc[P], xc[P], l2c[P], d2c[P], x2c[P];
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        lc[q] = l[q];
                        dc[q] = d[q];
                        xc[q] = x[q];
                        l2c[q] = s2_c == s_c ? l[q] : l2[q];
                        d2c[q] = s2_c == s_c ? d[q] : d2[q];
                        x2c[q] = s2_c == s_c ? x[q] : x2[q];
                    }
                    idx += EV;
                    if (idx < end) fetch(idx);
                    if (!act_c) continue;
                    if (kind_c == 0) {
                        const uint32_t ch = lat_reaction<P, BC, CU, CA, CI>(lc, dc, xc, a,
                                                                            (uint32_t)w, e_c, act_c);
                        if (ch) store_at(s_c, lc, dc, xc);
                        n_real += __popc(ch);
                    } else {
                        uint32_t mv, bl;
                        lat_hop<P>(s2_c == s_c, lc, dc, xc, l2c, d2c, x2c, a, (uint32_t)w, e_c,
                                   act_c, mv, bl);
                        if (mv) {
                            store_at(s_c, lc, dc, xc);
                            store_at(s2_c, l2c, d2c, x2c);
                        }
                        n_real += __popc(mv);
                        n_blocked += __popc(bl);
                    }
                }
                __syncthreads();
            }
        }
    }
    if (ST > 0 && runs) {
        __syncthreads();
        for (uint32_t k = tid; k < 3 * WS * nst; k += BLOCK)
            reinterpret_cast<uint4 *>(
                site_planes(a.planes, w0 + (k / 3) % WS, k / (3 * WS), S, NP))[k % 3] = stage[k];
    }
    // per-word totals of real events and blocked hops
    if (n_real) atomicAdd(&sred[0][lw], n_real);
    if (n_blocked) atomicAdd(&sred[1][lw], n_blocked);
    __syncthreads();
    if (tid < WS && w < words) {
        a.real[w] += sred[0][tid];
        a.blocked[w] += sred[1][tid];
    }
}

// ---- readouts --------------------------------------------------------------

// Species totals over sites of every replica: dst[i*3 + x].  A workgroup
// takes one word (the piece of the launch starts at word w0): thread t reads
// lane t mod 32 of the word on every LAT_TOT_SPLIT-th site from t / 32, so a
// half-wave reads one site's planes once for its 32 lanes and the sites of a
// word are read in parallel; the partial sums meet in LDS.
constexpr int LAT_TOT_SPLIT = 8;

template <int P>
__global__ __launch_bounds__(32 * LAT_TOT_SPLIT) void lat_totals_kernel(const uint32_t *planes,
                                                                        uint64_t M, int S,
                                                                        int32_t *dst, uint64_t w0)
{
    __shared__ int32_t part[LAT_TOT_SPLIT][3][32];
    const uint64_t w = w0 + blockIdx.x;
    const uint32_t lane = threadIdx.x & 31, sub = threadIdx.x >> 5;
    int32_t t[3] = {0, 0, 0};
    // several sites' loads in flight per thread
#pragma unroll 4
    for (int s = (int)sub; s < S; s += LAT_TOT_SPLIT) {
        uint32_t l[P], d[P], x[P];
        load_site<P>(site_planes(planes, w, (uint32_t)s, S, 3 * P), l, d, x);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            t[0] += (int32_t)((l[q] >> lane) & 1u) << q;
            t[1] += (int32_t)((d[q] >> lane) & 1u) << q;
            t[2] += (int32_t)((x[q] >> lane) & 1u) << q;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) part[sub][k][lane] = t[k];
    __syncthreads();
    if (threadIdx.x < 96) {
        const uint32_t k = threadIdx.x / 32, r = threadIdx.x % 32;
        int32_t v = 0;
#pragma unroll
        for (int j = 0; j < LAT_TOT_SPLIT; ++j) v += part[j][k][r];
        const uint64_t i = 32 * w + r;
        if (i < M) dst[3 * i + k] = v;
    }
}

// Site counts of replicas first .. first+count-1: dst[(k S + s) 3 + x].
__global__ void lat_sites_kernel(const uint32_t *planes, int S, int P, uint64_t first,
                                 uint64_t count, int32_t *dst)
{
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t s = blockIdx.y;
    if (k >= count) return;
    const uint64_t i = first + k;
    const uint64_t w = i >> 5;
    const uint32_t lane = i & 31;
    const uint32_t *p = site_planes(planes, w, s, S, 3 * P);
    for (int x = 0; x < 3; ++x) {
        int32_t v = 0;
        for (int q = 0; q < P; ++q) v |= (int32_t)((p[x * P + q] >> lane) & 1u) << q;
        dst[(k * S + s) * 3 + x] = v;
    }
}

// ee histogram from per-replica totals: n = L + D + A of the replica,
// bin = min(n_bins - 1, (L - D + n) n_bins / (2 n)), n = 0 in bin n_bins / 2.
__global__ void lat_histogram_kernel(const int32_t *tot, uint64_t M, int n_bins, uint64_t *dst)
{
    extern __shared__ uint32_t h[];
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t L = tot[3 * i], D = tot[3 * i + 1], A = tot[3 * i + 2];
        const int64_t n = L + D + A;
        int64_t b = n_bins / 2;
        if (n > 0) b = min((int64_t)n_bins - 1, ((L - D + n) * n_bins) / (2 * n));
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (h[b]) atomicAdd((unsigned long long *)&dst[b], (unsigned long long)h[b]);
}

// ---- launchers ---------------------------------------------------------------

hipError_t launch_lat_init(uint32_t *planes, uint64_t words, uint64_t M, int S, int P, int mode,
                           const int32_t *sites_dev, const int32_t c3[3], int32_t lo, int32_t hi,
                           uint64_t seed, uint32_t net_id, uint64_t *E, uint64_t *Et,
                           uint64_t *real, uint64_t *blocked, hipStream_t s)
{
    if (mode == 0) {
        dim3 grid((unsigned)((words + 255) / 256), (unsigned)S);
        hipLaunchKernelGGL(lat_init_fixed_kernel, grid, dim3(256), 0, s, planes, words, M, S, P,
                           sites_dev, c3[0], c3[1], c3[2], E, Et, real, blocked);
    } else {
        const uint64_t reps = 64 * ((words + 1) / 2);
        dim3 grid((unsigned)((reps + 255) / 256), (unsigned)S);
        hipLaunchKernelGGL(lat_init_uniform_kernel, grid, dim3(256), 0, s, planes, words, M, S, P,
                           lo, hi, seed, net_id, E, Et, real, blocked);
    }
    return hipGetLastError();
}

hipError_t launch_lat_schedule(const LatArgs &a, uint32_t n_groups, hipStream_t s)
{
    hipLaunchKernelGGL(lat_schedule_kernel, dim3(n_groups * a.n_chunks), dim3(64), 0, s, a);
    return hipGetLastError();
}

// (id, P, BC, CU, CA, CI, WS, BLOCK, ST): species planes, threshold-plane
// capacity, the weights of A -> L / A -> D, A + L -> 2L / A + D -> 2D and
// L + D -> 2A (-1: taken at run time), words per slice, threads per
// workgroup (512 for the run-time weights, which need more registers) and
// sites staged in LDS (0: none).
#define BWG_LAT_VARIANTS(X)                                                                   \
    X(0, 4, 19, 246, 2048, 2048, 4, 1024, 0) X(1, 4, 19, 246, 2048, 2048, 1, 1024, 0)          \
    X(2, 4, 19, -1, -1, -1, 4, 512, 0) X(3, 4, 19, -1, -1, -1, 1, 512, 0)                      \
    X(4, 4, 24, -1, -1, -1, 4, 512, 0) X(5, 4, 24, -1, -1, -1, 1, 512, 0)                      \
    X(6, 4, 19, 246, 2048, 2048, 4, 1024, 4 * BWG_LAT_STAGE_SITES)

// grid: the slices of the band's groups, rounded up to a multiple of the 8 XCDs
#define BWG_LAT_LAUNCH(ID, P_, BC_, CU_, CA_, CI_, WS_, BL_, ST_)                             \
    static hipError_t lat_launch_##ID(const LatArgs &a, uint64_t words, hipStream_t s)       \
    {                                                                                         \
        (void)words;                                                                          \
        const uint64_t nwg = (uint64_t)a.ng * (LAT_GROUP_WORDS / WS_);                        \
        hipLaunchKernelGGL((lat_event_kernel<P_, BC_, CU_, CA_, CI_, WS_, BL_, ST_>),         \
                           dim3((unsigned)(8 * ((nwg + 7) / 8))), dim3(BL_), 0, s, a);        \
        return hipGetLastError();                                                             \
    }
BWG_LAT_VARIANTS(BWG_LAT_LAUNCH)

#ifndef __HIP_DEVICE_COMPILE__
#define BWG_LAT_ROW(ID, P_, BC_, CU_, CA_, CI_, WS_, BL_, ST_) {P_, BC_, CU_, CA_, CI_, WS_, BL_, ST_, lat_launch_##ID},
const LatVariant kLatVariants[] = {BWG_LAT_VARIANTS(BWG_LAT_ROW)};
const int kLatVariantCount = sizeof(kLatVariants) / sizeof(kLatVariants[0]);
#endif

hipError_t launch_lat_totals(const uint32_t *planes, uint64_t M, int S, int P, int32_t *dst,
                             hipStream_t s)
{
    if (P != 4) return hipErrorInvalidValue;
    // one workgroup per word
    constexpr uint32_t block = 32 * LAT_TOT_SPLIT;
    return launch_pieces((M + 31) / 32 * block, block, [&](uint64_t i0, dim3 g) {
        hipLaunchKernelGGL(lat_totals_kernel<4>, g, dim3(block), 0, s, planes, M, S, dst,
                           i0 / block);
    });
}

hipError_t launch_lat_sites(const uint32_t *planes, int S, int P, uint64_t first, uint64_t count,
                            int32_t *dst, hipStream_t s)
{
    dim3 grid((unsigned)((count + 255) / 256), (unsigned)S);
    hipLaunchKernelGGL(lat_sites_kernel, grid, dim3(256), 0, s, planes, S, P, first, count, dst);
    return hipGetLastError();
}

hipError_t launch_lat_histogram(const int32_t *tot, uint64_t M, int n_bins, uint64_t *dst,
                                hipStream_t s)
{
    hipError_t err = launch_fill_u64(dst, (uint64_t)n_bins, 0, s);
    if (err != hipSuccess) return err;
    const unsigned blocks = (unsigned)std::min<uint64_t>(1024, (M + 255) / 256);
    hipLaunchKernelGGL(lat_histogram_kernel, dim3(blocks), dim3(256), n_bins * 4, s, tot, M,
                       n_bins, dst);
    return hipGetLastError();
}

}  // namespace bwg
