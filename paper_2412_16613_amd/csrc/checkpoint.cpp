// Checkpoint and resume of an ensemble between advances.
//
// Every draw of the chain is keyed by the replica, the absolute event index
// and the advance index (counter-based Philox), so the state that fixes the
// rest of a run is the per-replica counts (bit planes or int32 counts), the
// event counters, the clock t_now and the advance index; real events and
// blocked hops are running statistics.  A checkpoint holds exactly these;
// the host bounds the kernels use (how far a word's lanes are apart, the
// lowest and highest event index of a lattice, the lockstep event of a
// shared-threshold ensemble) are derived again from the restored counters.

#include <string.h>

#include <algorithm>

#include "host_internal.h"

using namespace bwg;

namespace {

constexpr uint64_t kMagic = 0x31544b5043475742ull;  // "BWGCPKT1", little-endian
constexpr uint64_t kHeaderWords = 32;
constexpr uint64_t kHeaderBytes = kHeaderWords * 8;
constexpr int kMaxRegions = 6;
// headroom below the 48 bits of event index the EVENT draw keys
constexpr uint64_t kMaxRestoredEvent = 1ull << 47;

enum : uint64_t { REG_PLANES = 1, REG_COUNTS = 2, REG_E = 3, REG_ET = 4, REG_REAL = 5,
                  REG_BLOCKED = 6 };
enum : uint64_t { KIND_PLANES = 0, KIND_PLAIN = 1, KIND_LATTICE = 2 };

struct Region {
    uint64_t id;
    void *dev;
    uint64_t bytes;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// FNV-1a over the integer form of the network: species and reaction tables,
// the quantised weights and scales, and for lattices their shape and weights.
struct Fnv {
    uint64_t h = 0xcbf29ce484222325ull;
    void add(const void *p, size_t n)
    {
        const uint8_t *b = (const uint8_t *)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 0x100000001b3ull;
        }
    }
    template <class T> void val(T v) { add(&v, sizeof v); }
};

uint64_t fingerprint(const bwg_net *n)
{
    Fnv f;
    f.val(n->S);
    f.val(n->R);
    f.add(n->reac.data(), n->reac.size() * sizeof(int32_t));
    f.add(n->prod.data(), n->prod.size() * sizeof(int32_t));
    f.val(n->n_tot);
    f.val((int32_t)n->open);
    f.val(n->lx);
    f.val(n->ly);
    for (int j = 0; j < n->R; ++j) f.val(n->q.c[j]);
    f.val(n->q.f);
    f.val(n->q.B);
    f.val(n->q.b);
    f.val(n->q.s);
    f.val(n->q.max_total);
    if (n->lat) {
        f.val(n->lsh.S);
        f.val(n->lsh.P);
        f.val(n->lsh.B_r);
        for (int j = 0; j < 5; ++j) f.val(n->c_lat[j]);
        f.val(n->c_hop);
        f.val(n->T);
    }
    return f.h;
}

uint64_t state_kind(const bwg_ens *e)
{
    if (e->lat) return KIND_LATTICE;
    return e->engine == BWG_ENGINE_PLAIN ? KIND_PLAIN : KIND_PLANES;
}

// The device regions that carry the ensemble's state, in checkpoint order.
int regions(const bwg_ens *e, Region *r)
{
    const bwg_net *n = e->net;
    int k = 0;
    if (e->lat) {
        const uint64_t mp = 32 * e->words;
        r[k++] = {REG_PLANES, e->planes,
                  e->groups * LAT_GROUP_WORDS * (uint64_t)n->lsh.S * 3 * n->lsh.P * 4};
        r[k++] = {REG_E, e->E, mp * 8};
        r[k++] = {REG_ET, e->Et, mp * 8};
        r[k++] = {REG_REAL, e->real, e->words * 8};
        r[k++] = {REG_BLOCKED, e->blocked, e->words * 8};
        return k;
    }
    const uint64_t mp = 32 * e->wp;
    if (e->engine == BWG_ENGINE_PLAIN)
        r[k++] = {REG_COUNTS, e->counts, 3 * mp * 4};
    else
        r[k++] = {REG_PLANES, e->planes, (uint64_t)n->S * e->nb * e->wp * 4};
    r[k++] = {REG_E, e->E, mp * 8};
    r[k++] = {REG_ET, e->Et, mp * 8};
    r[k++] = {REG_REAL, e->real, (e->engine == BWG_ENGINE_PLAIN ? mp : e->wp) * 8};
    return k;
}

uint64_t total_bytes(const Region *r, int k)
{
    uint64_t off = kHeaderBytes;
    for (int i = 0; i < k; ++i) off = align256(off) + r[i].bytes;
    return off;
}

}  // namespace

extern "C" int bwg_ensemble_checkpoint_bytes(const bwg_ens *e, uint64_t *bytes)
{
    if (!e || !bytes) return fail(BWG_EINVAL, "null argument");
    Region r[kMaxRegions];
    *bytes = total_bytes(r, regions(e, r));
    return BWG_OK;
}

extern "C" int bwg_ensemble_save(bwg_ens *e, void *host_dst, uint64_t dst_bytes, void *stream)
{
    TraceRange trace_("bwg_ensemble_save");
    if (!e || !host_dst) return fail(BWG_EINVAL, "null argument");
    if (!e->inited) return fail(BWG_EINVAL, "ensemble not initialised");
    if (e->pending)
        return fail(BWG_EINVAL, "events of the last advance are still pending (save between "
                                "advances)");
    Region r[kMaxRegions];
    const int k = regions(e, r);
    const uint64_t need = total_bytes(r, k);
    if (dst_bytes < need)
        return fail(BWG_ERANGE, "checkpoint needs %llu bytes, buffer holds %llu",
                    (unsigned long long)need, (unsigned long long)dst_bytes);
    hipStream_t s = (hipStream_t)stream;
    uint8_t *dst = (uint8_t *)host_dst;
    uint64_t h[kHeaderWords] = {};
    h[0] = kMagic;
    h[1] = kHeaderBytes;
    h[2] = need;
    h[3] = fingerprint(e->net);
    h[4] = e->M;
    h[5] = e->seed;
    h[6] = e->net_id;
    h[7] = state_kind(e);
    h[8] = e->zs;
    memcpy(&h[9], &e->t_now, 8);
    h[10] = e->adv;
    h[11] = (uint64_t)k;
    uint64_t off = kHeaderBytes;
    for (int i = 0; i < k; ++i) {
        off = align256(off);
        h[12 + 3 * i] = r[i].id;
        h[13 + 3 * i] = off;
        h[14 + 3 * i] = r[i].bytes;
        HIP_TRY(hipMemcpyAsync(dst + off, r[i].dev, r[i].bytes, hipMemcpyDeviceToHost, s));
        off += r[i].bytes;
    }
    memcpy(dst, h, sizeof h);
    HIP_TRY(hipStreamSynchronize(s));
    return BWG_OK;
}

extern "C" int bwg_ensemble_restore(bwg_ens *e, const void *host_src, uint64_t src_bytes,
                                    void *stream)
{
    TraceRange trace_("bwg_ensemble_restore");
    if (!e || !host_src) return fail(BWG_EINVAL, "null argument");
    if (e->pending)
        return fail(BWG_EINVAL, "events of the last advance are still pending");
    if (src_bytes < kHeaderBytes) return fail(BWG_EINVAL, "not a checkpoint (too short)");
    const uint8_t *src = (const uint8_t *)host_src;
    uint64_t h[kHeaderWords];
    memcpy(h, src, sizeof h);
    if (h[0] != kMagic || h[1] != kHeaderBytes) return fail(BWG_EINVAL, "not a checkpoint");
    Region r[kMaxRegions];
    const int k = regions(e, r);
    const uint64_t need = total_bytes(r, k);
    if (h[2] != need || src_bytes < need)
        return fail(BWG_EINVAL, "checkpoint of %llu bytes, this ensemble's takes %llu",
                    (unsigned long long)h[2], (unsigned long long)need);
    if (h[3] != fingerprint(e->net))
        return fail(BWG_EINVAL, "checkpoint of another network");
    if (h[4] != e->M)
        return fail(BWG_EINVAL, "checkpoint of %llu replicas, ensemble of %llu",
                    (unsigned long long)h[4], (unsigned long long)e->M);
    if (h[7] != state_kind(e))
        return fail(BWG_EINVAL, "checkpoint of another state kind (bit planes, plain counts, "
                                "lattice)");
    if (h[8] != e->zs)
        return fail(BWG_EINVAL, "checkpoint and ensemble differ in the shared threshold");
    if (h[11] != (uint64_t)k) return fail(BWG_EINVAL, "checkpoint regions do not match");
    // the counters are read with memcpy: the caller's buffer need not be
    // 8-byte aligned
    const uint8_t *E = nullptr, *Et = nullptr;
    for (int i = 0; i < k; ++i) {
        const uint64_t id = h[12 + 3 * i], off = h[13 + 3 * i], bytes = h[14 + 3 * i];
        if (id != r[i].id || bytes != r[i].bytes || off % 256 || off > need ||
            bytes > need - off)
            return fail(BWG_EINVAL, "checkpoint regions do not match");
        if (id == REG_E) E = src + off;
        if (id == REG_ET) Et = src + off;
    }
    // between advances every replica has run its budget; derive the host
    // bounds from the live replicas' counters
    uint64_t lo = ~0ull, hi = 0, lag = 0;
    const uint64_t words = (e->M + 31) / 32;
    for (uint64_t w = 0; w < words; ++w) {
        uint64_t wlo = ~0ull, whi = 0;
        const uint64_t end = std::min<uint64_t>(32 * w + 32, e->M);
        for (uint64_t i = 32 * w; i < end; ++i) {
            uint64_t ei, ti;
            memcpy(&ei, E + 8 * i, 8);
            memcpy(&ti, Et + 8 * i, 8);
            if (ei != ti)
                return fail(BWG_EINVAL, "replica %llu has pending events in the checkpoint",
                            (unsigned long long)i);
            wlo = std::min(wlo, ei);
            whi = std::max(whi, ei);
        }
        lo = std::min(lo, wlo);
        hi = std::max(hi, whi);
        lag = std::max(lag, whi - wlo);
    }
    if (hi >= kMaxRestoredEvent)
        return fail(BWG_ERANGE, "event index %llu beyond 2^47", (unsigned long long)hi);
    if (e->zs && lo != hi)
        return fail(BWG_EINVAL, "shared-threshold replicas must stand at one event");
    double t_now;
    memcpy(&t_now, &h[9], 8);
    if (!(t_now >= 0) || h[10] >= (1ull << 48))
        return fail(BWG_EINVAL, "checkpoint clock out of range");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < k; ++i)
        HIP_TRY(hipMemcpyAsync(r[i].dev, src + h[13 + 3 * i], r[i].bytes, hipMemcpyHostToDevice,
                               s));
    HIP_TRY(launch_fill_u64(e->adv_dev, 1, h[10], s));
    HIP_TRY(hipStreamSynchronize(s));
    e->t_now = t_now;
    e->adv = h[10];
    e->pending = 0;
    e->lag = lag;
    e->zE = lo;
    e->zbase = e->zlen = 0;   // shared thresholds are drawn again from zE
    e->emin = lo;
    e->emax = hi;
    e->base = e->n_chunks = e->cursor = 0;
    e->inited = true;
    return BWG_OK;
}
