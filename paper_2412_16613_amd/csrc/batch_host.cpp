// C ABI of batches: many ensembles whose pending events run in one
// persistent launch; membership can change between launches (continuous
// batching), and one batch advance can be captured in a graph and replayed.

#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "host_internal.h"

using namespace bwg;

struct bwg_batch {
    std::vector<bwg_ens *> ens;
    std::vector<int> bucket;       // persistent-kernel plane bucket per member
    std::vector<double> cost;      // issue cost of one event of a 64-word item, per member
    std::vector<double> lane_cost; // the same for a 2-word lanes item
    int waves = 0;
    int order = 0;
    int cap_ens = 0;
    uint64_t cap_items = 0;
    uint64_t n_items = 0;          // items of the current members
    bool lanes_items = false;      // the staged queue holds lanes items
    // device layout (caller buffer)
    BatchEns *d_ens = nullptr;
    BatchBudget *d_budget = nullptr;
    BatchItem *d_items = nullptr;
    uint32_t *d_counter = nullptr;
    // pinned staging and the event that guards its reuse
    BatchEns *h_ens = nullptr;
    BatchBudget *h_budget = nullptr;
    BatchItem *h_items = nullptr;
    uint64_t *h_tables = nullptr;  // Poisson tables of an advance, back to back
    uint64_t h_tables_cap = 0;     // entries
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    ~bwg_batch()
    {
        if (staged_pending) (void)hipEventSynchronize(staged);
        if (staged) (void)hipEventDestroy(staged);
        if (h_ens) (void)hipHostFree(h_ens);
        if (h_budget) (void)hipHostFree(h_budget);
        if (h_items) (void)hipHostFree(h_items);
        if (h_tables) (void)hipHostFree(h_tables);
    }
};

static uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

static int pick_bucket(const bwg_ens *e)
{
    const bwg_net *n = e->net;
    const int need_bc = n->q.B + (n->q.max_total == (1ll << n->q.B) ? 1 : 0);
    int best = -1;
    for (int i = 0; i < kPersistVariantCount; ++i) {
        const PersistVariant &v = kPersistVariants[i];
        if (v.nb < n->q.b || v.bc < need_bc) continue;
        if (n->shape.fa >= v.bc || n->shape.fi >= v.bc) continue;
        if (best < 0 || v.nb + v.bc < kPersistVariants[best].nb + kPersistVariants[best].bc)
            best = i;
    }
    return best < 0 ? -1 : kPersistVariants[best].id;
}

// Work items of a member: words [0, split) in items of 64 (one word per
// lane, bit-sliced), words [split, words) in items of 2 (one per half wave,
// one replica per lane: the lanes engine).  split is 0 for members on the
// lanes engine and a multiple of 64 otherwise.
static uint64_t lanes_split(const bwg_ens *e)
{
    const uint64_t words = (e->M + 31) / 32;
    if (e->engine == BWG_ENGINE_LANES) return 0;
    if (e->lanes_words >= words) return 0;
    return (words - e->lanes_words + 63) / 64 * 64;
}
static uint64_t n_items_of(const bwg_ens *e)
{
    const uint64_t words = (e->M + 31) / 32, split = std::min(lanes_split(e), words);
    return (split + 63) / 64 + (words - split + 1) / 2;
}

static uint64_t layout_bytes(int n, uint64_t items, uint64_t *off_ens, uint64_t *off_budget,
                             uint64_t *off_items, uint64_t *off_counter)
{
    uint64_t o = 0;
    *off_ens = o;
    o = a256(o + sizeof(BatchEns) * (uint64_t)n);
    *off_budget = o;
    o = a256(o + sizeof(BatchBudget) * (uint64_t)n);
    *off_items = o;
    o = a256(o + sizeof(BatchItem) * items);
    *off_counter = o;
    o = a256(o + 64);
    return o;
}

static int check_members(bwg_ens *const *ens, int32_t n, uint64_t *items)
{
    if (n < 0 || (n > 0 && !ens)) return fail(BWG_EINVAL, "bad member list");
    uint64_t it = 0;
    for (int k = 0; k < n; ++k) {
        const bwg_ens *e = ens[k];
        if (!e) return fail(BWG_EINVAL, "null ensemble %d", k);
        if (e->engine != BWG_ENGINE_BITWISE && e->engine != BWG_ENGINE_LANES)
            return fail(BWG_EUNSUPPORTED, "ensemble %d: batches run the bit-plane engines", k);
        if (e->zs)
            return fail(BWG_EUNSUPPORTED, "ensemble %d: shared-threshold ensembles move by step", k);
        if (!e->net->shape_ok)
            return fail(BWG_EUNSUPPORTED, "ensemble %d: batches run Frank-family networks", k);
        if (e->lat)
            return fail(BWG_EUNSUPPORTED, "ensemble %d: lattices run their own launches", k);
        if (pick_bucket(e) < 0)
            return fail(BWG_EUNSUPPORTED, "ensemble %d: no persistent bucket for b=%d B=%d", k,
                        e->net->q.b, e->net->q.B);
        for (int j = 0; j < k; ++j)
            if (ens[j] == e) return fail(BWG_EINVAL, "ensemble %d appears twice", k);
        it += n_items_of(e);
    }
    if (it >= (1ull << 32)) return fail(BWG_ERANGE, "too many work items");
    *items = it;
    return BWG_OK;
}

extern "C" int bwg_batch_state_bytes(bwg_ens *const *ens, int32_t n, uint64_t *bytes)
{
    if (!bytes) return fail(BWG_EINVAL, "null argument");
    uint64_t items;
    int rc = check_members(ens, n, &items);
    if (rc) return rc;
    uint64_t a, b, c, d;
    *bytes = layout_bytes(n, items, &a, &b, &c, &d);
    return BWG_OK;
}

extern "C" int bwg_batch_capacity_bytes(int32_t max_ensembles, uint64_t max_items, uint64_t *bytes)
{
    if (!bytes || max_ensembles < 1) return fail(BWG_EINVAL, "bad capacity");
    uint64_t a, b, c, d;
    *bytes = layout_bytes(max_ensembles, max_items, &a, &b, &c, &d);
    return BWG_OK;
}

static hipError_t sync_staging(bwg_batch *b)
{
    if (!b->staged_pending) return hipSuccess;
    b->staged_pending = false;
    return hipEventSynchronize(b->staged);
}

// Install members: descriptors of every member, uploaded on the stream.
static int set_members(bwg_batch *b, bwg_ens *const *ens, int32_t n, hipStream_t s)
{
    uint64_t items;
    int rc = check_members(ens, n, &items);
    if (rc) return rc;
    if (n > b->cap_ens || items > b->cap_items)
        return fail(BWG_ERANGE, "%d members / %llu items exceed the batch capacity %d / %llu", n,
                    (unsigned long long)items, b->cap_ens, (unsigned long long)b->cap_items);
    HIP_TRY(sync_staging(b));
    b->ens.assign(ens, ens + n);
    b->bucket.clear();
    b->cost.clear();
    b->lane_cost.clear();
    b->n_items = items;
    for (int k = 0; k < n; ++k) {
        const bwg_ens *e = ens[k];
        const bwg_net *nt = e->net;
        const int bk = pick_bucket(e);
        b->bucket.push_back(bk);
        const PersistVariant &v = kPersistVariants[bk];
        // per-event issue cost of one item (orders the queue only): a lanes
        // item's event takes ~50 instructions plus its share of the draws and
        // the transposition of 32 events' planes
        b->cost.push_back(100.0 * ((nt->q.B + 3) / 4) + 8.0 * v.bc + 40.0 * v.nb);
        b->lane_cost.push_back(60.0 + 1.5 * nt->q.B);
        BatchEns &d = b->h_ens[k];
        memset(&d, 0, sizeof d);
        WmArgs &a = d.a;
        a.planes = e->planes;
        a.E = e->E;
        a.Etgt = e->Et;
        a.real = e->real;
        a.wp = e->wp;
        a.n_words = (e->M + 31) / 32;
        a.M = e->M;
        a.seed = e->seed;
        a.max_events = 0;
        a.net_id = e->net_id;
        a.B = nt->q.B;
        a.cu = nt->shape.cu;
        a.fa = nt->shape.fa;
        a.fi = nt->shape.fi;
        a.nb_mem = e->nb;
        d.variant = bk;
    }
    if (n)
        HIP_TRY(hipMemcpyAsync(b->d_ens, b->h_ens, sizeof(BatchEns) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(b->staged, s));
    b->staged_pending = true;
    return BWG_OK;
}

extern "C" int bwg_batch_create(bwg_ens *const *ens, int32_t n, void *dev_buf, uint64_t buf_bytes,
                                const bwg_batch_opts *opts, void *stream, bwg_batch **out)
{
    TraceRange trace_("bwg_batch_create");
    if (!out || !dev_buf) return fail(BWG_EINVAL, "null argument");
    *out = nullptr;
    if ((uintptr_t)dev_buf & 255) return fail(BWG_EINVAL, "device buffer not 256-byte aligned");
    uint64_t items;
    int rc = check_members(ens, n, &items);
    if (rc) return rc;
    const int cap_ens = std::max<int>(n, opts ? opts->max_ensembles : 0);
    const uint64_t cap_items = std::max<uint64_t>(items, opts ? opts->max_items : 0);
    if (cap_ens < 1) return fail(BWG_EINVAL, "empty batch without capacity");
    uint64_t o_ens, o_bud, o_it, o_cnt;
    const uint64_t need = layout_bytes(cap_ens, cap_items, &o_ens, &o_bud, &o_it, &o_cnt);
    if (buf_bytes < need)
        return fail(BWG_ENOMEM, "batch buffer of %llu bytes, need %llu",
                    (unsigned long long)buf_bytes, (unsigned long long)need);
    auto b = new bwg_batch();
    b->waves = (opts && opts->waves > 0) ? opts->waves : 2048;
    b->order = opts ? opts->order : 0;
    b->cap_ens = cap_ens;
    b->cap_items = cap_items;
    uint8_t *base = (uint8_t *)dev_buf;
    b->d_ens = (BatchEns *)(base + o_ens);
    b->d_budget = (BatchBudget *)(base + o_bud);
    b->d_items = (BatchItem *)(base + o_it);
    b->d_counter = (uint32_t *)(base + o_cnt);
    if (hipHostMalloc((void **)&b->h_ens, sizeof(BatchEns) * cap_ens, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&b->h_budget, sizeof(BatchBudget) * cap_ens, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&b->h_items, sizeof(BatchItem) * std::max<uint64_t>(cap_items, 1),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(BWG_EDEVICE, "pinned staging allocation failed");
    }
    rc = set_members(b, ens, n, (hipStream_t)stream);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return BWG_OK;
}

extern "C" int bwg_batch_set_members(bwg_batch *b, bwg_ens *const *ens, int32_t n, void *stream)
{
    TraceRange trace_("bwg_batch_set_members");
    if (!b) return fail(BWG_EINVAL, "null batch");
    return set_members(b, ens, n, (hipStream_t)stream);
}

extern "C" void bwg_batch_destroy(bwg_batch *b) { delete b; }

// Queue of the members' items, longest pending work first (or in member
// order), uploaded on the stream.
static int stage_items(bwg_batch *b, hipStream_t s)
{
    std::vector<std::pair<double, BatchItem>> q;
    q.reserve(b->n_items);
    b->lanes_items = false;
    for (size_t k = 0; k < b->ens.size(); ++k) {
        const bwg_ens *e = b->ens[k];
        const uint64_t words = (e->M + 31) / 32, split = std::min(lanes_split(e), words);
        const double cw = b->cost[k] * (double)e->pending;
        const double cl = b->lane_cost[k] * (double)e->pending;
        for (uint64_t w0 = 0; w0 < split; w0 += 64)
            q.push_back({cw, BatchItem{(uint32_t)k, (uint32_t)w0}});
        for (uint64_t w0 = split; w0 < words; w0 += 2)
            q.push_back({cl, BatchItem{(uint32_t)k | BATCH_ITEM_LANES, (uint32_t)w0}});
        if (split < words) b->lanes_items = true;
    }
    if (b->order == 0)
        std::stable_sort(q.begin(), q.end(),
                         [](const std::pair<double, BatchItem> &x,
                            const std::pair<double, BatchItem> &y) { return x.first > y.first; });
    for (size_t i = 0; i < q.size(); ++i) b->h_items[i] = q[i].second;
    if (!q.empty())
        HIP_TRY(hipMemcpyAsync(b->d_items, b->h_items, sizeof(BatchItem) * q.size(),
                               hipMemcpyHostToDevice, s));
    return BWG_OK;
}

// Tables and budget descriptors of one advance of every member to t_end[k].
// The members' Poisson tables (binary128 sums, up to a few ms each for long
// horizons) are built on up to 16 host threads, then staged back to back in
// the batch's pinned buffer (reused once its last upload has completed).
static int stage_budgets(bwg_batch *b, const double *t_end, hipStream_t s,
                         std::vector<uint64_t> &kmin, std::vector<uint64_t> &kmax)
{
    const int n = (int)b->ens.size();
    kmin.assign(n, 0);
    kmax.assign(n, 0);
    std::vector<double> mu(n, 0.0);
    int need = 0;
    for (int k = 0; k < n; ++k) {
        const bwg_ens *e = b->ens[k];
        if (!e->inited) return fail(BWG_EINVAL, "ensemble %d not initialised", k);
        if (!(t_end[k] >= e->t_now))
            return fail(BWG_EINVAL, "ensemble %d: t_end %g before t_now %g", k, t_end[k], e->t_now);
        mu[k] = e->net->q.lambda * (t_end[k] - e->t_now);
        if (mu[k] > 0) ++need;
    }
    std::vector<const Table *> tab(n, nullptr);
    std::vector<int> rc(n, BWG_OK);
    std::vector<std::string> msg(n);
    std::atomic<int> next(0);
    auto work = [&]() {
        for (int k; (k = next.fetch_add(1)) < n;) {
            if (!(mu[k] > 0)) continue;
            rc[k] = get_table(b->ens[k]->net, mu[k], &tab[k], false);
            if (rc[k]) msg[k] = bwg_last_error();
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::min<int>(need, (int)std::min(16u, hw));
    std::vector<std::thread> pool;
    for (int i = 1; i < nt; ++i) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
    uint64_t total = 0;
    for (int k = 0; k < n; ++k) {
        if (rc[k]) return fail(rc[k], "ensemble %d: %s", k, msg[k].c_str());
        if (!tab[k]) continue;
        if (tab[k]->len > b->ens[k]->table_cap)
            return fail(BWG_ERANGE, "ensemble %d: Poisson table of %llu entries exceeds %llu", k,
                        (unsigned long long)tab[k]->len,
                        (unsigned long long)b->ens[k]->table_cap);
        total += tab[k]->len;
    }
    if (total > b->h_tables_cap) {
        if (b->h_tables) HIP_TRY(hipHostFree(b->h_tables));
        b->h_tables = nullptr;
        b->h_tables_cap = 0;
        const uint64_t cap = total + total / 4;
        HIP_TRY(hipHostMalloc((void **)&b->h_tables, cap * sizeof(uint64_t), hipHostMallocDefault));
        b->h_tables_cap = cap;
    }
    uint64_t offset = 0, toff = 0;
    for (int k = 0; k < n; ++k) {
        bwg_ens *e = b->ens[k];
        BatchBudget &bb = b->h_budget[k];
        memset(&bb, 0, sizeof bb);
        if (const Table *t = tab[k]) {
            memcpy(b->h_tables + toff, t->vals.data(), t->len * sizeof(uint64_t));
            HIP_TRY(hipMemcpyAsync(e->table, b->h_tables + toff, t->len * 8, hipMemcpyHostToDevice,
                                   s));
            toff += t->len;
            bb.T = e->table;
            bb.len = t->len;
            bb.k_lo = t->k_lo;
            kmin[k] = (uint64_t)t->k_lo;
            kmax[k] = (uint64_t)t->k_lo + t->len;
        }
        bb.seed = e->seed;
        bb.offset = offset;
        bb.adv = e->adv_dev;
        bb.E = e->E;
        bb.Et = e->Et;
        bb.net_id = e->net_id;
        offset += e->M;
    }
    if (n)
        HIP_TRY(hipMemcpyAsync(b->d_budget, b->h_budget, sizeof(BatchBudget) * n,
                               hipMemcpyHostToDevice, s));
    return BWG_OK;
}

static uint64_t total_replicas(const bwg_batch *b)
{
    uint64_t t = 0;
    for (auto *e : b->ens) t += e->M;
    return t;
}

// Budget draws and advance-index increments of every member (kernels only).
static int enqueue_budgets(bwg_batch *b, hipStream_t s)
{
    const int n = (int)b->ens.size();
    if (!n) return BWG_OK;
    HIP_TRY(launch_batch_budget(b->d_budget, n, total_replicas(b), s));
    HIP_TRY(launch_batch_epilogue(b->d_budget, n, s));
    return BWG_OK;
}

// One persistent pass over the staged queue (kernels only).
static int enqueue_pass(bwg_batch *b, uint64_t max_events, hipStream_t s)
{
    if (!b->n_items) return BWG_OK;
    HIP_TRY(launch_batch_prologue(b->d_counter, s));
    HIP_TRY(launch_persistent(b->d_ens, b->d_items, (uint32_t)b->n_items, b->d_counter, b->waves,
                              max_events, b->lanes_items, s));
    return BWG_OK;
}

static void note_budgets(bwg_batch *b, const double *t_end, const std::vector<uint64_t> &kmin,
                         const std::vector<uint64_t> &kmax)
{
    for (size_t k = 0; k < b->ens.size(); ++k) {
        bwg_ens *e = b->ens[k];
        note_scheduled(e, kmin[k], kmax[k]);
        e->t_now = t_end[k];
        e->adv += 1;
    }
}

extern "C" int bwg_batch_advance(bwg_batch *b, const double *t_end, void *stream)
{
    TraceRange trace_("bwg_batch_advance");
    if (!b || (!t_end && !b->ens.empty())) return fail(BWG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(sync_staging(b));
    std::vector<uint64_t> kmin, kmax;
    int rc = stage_budgets(b, t_end, s, kmin, kmax);
    if (rc) return rc;
    rc = enqueue_budgets(b, s);
    if (rc) return rc;
    note_budgets(b, t_end, kmin, kmax);
    rc = stage_items(b, s);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b->staged, s));
    b->staged_pending = true;
    rc = enqueue_pass(b, 0, s);
    if (rc) return rc;
    for (auto *e : b->ens) note_ran(e, 0);
    return BWG_OK;
}

extern "C" int bwg_batch_run(bwg_batch *b, uint64_t max_events, void *stream)
{
    TraceRange trace_("bwg_batch_run");
    if (!b) return fail(BWG_EINVAL, "null batch");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(sync_staging(b));
    int rc = stage_items(b, s);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b->staged, s));
    b->staged_pending = true;
    rc = enqueue_pass(b, max_events, s);
    if (rc) return rc;
    for (auto *e : b->ens) note_ran(e, max_events);
    return BWG_OK;
}

extern "C" int bwg_batch_graph_advance(bwg_batch *b, double dt, int32_t n_steps, void *stream)
{
    TraceRange trace_("bwg_batch_graph_advance");
    if (!b) return fail(BWG_EINVAL, "null batch");
    if (n_steps < 1 || !(dt >= 0)) return fail(BWG_EINVAL, "need n_steps >= 1 and dt >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(BWG_EINVAL, "graph capture needs a non-null stream");
    const size_t n = b->ens.size();
    // every step must have the same mean: (t + dt) - t == dt exactly
    for (size_t k = 0; k < n; ++k) {
        double t = b->ens[k]->t_now;
        for (int i = 0; i < n_steps; ++i) {
            const double t2 = t + dt;
            if (t2 - t != dt)
                return fail(BWG_EINVAL, "ensemble %zu: step %d of %g is not exact in binary64", k,
                            i, dt);
            t = t2;
        }
    }
    HIP_TRY(sync_staging(b));
    std::vector<double> t_end(n);
    for (size_t k = 0; k < n; ++k) t_end[k] = b->ens[k]->t_now + dt;
    std::vector<uint64_t> kmin, kmax;
    int rc = stage_budgets(b, t_end.data(), s, kmin, kmax);
    if (rc) return rc;
    // the queue order of the first step serves every replay
    for (size_t k = 0; k < n; ++k) b->ens[k]->pending = b->ens[k]->lag + kmax[k];
    rc = stage_items(b, s);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b->staged, s));
    b->staged_pending = true;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = enqueue_budgets(b, s);
    if (!rc) rc = enqueue_pass(b, 0, s);
    hipError_t ce = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ce != hipSuccess) return fail(BWG_EDEVICE, "graph capture: %s", hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(BWG_EDEVICE, "graph instantiation: %s", hipGetErrorString(ie));
    }
    int err = BWG_OK;
    for (int i = 0; i < n_steps; ++i) {
        hipError_t le = hipGraphLaunch(ge, s);
        if (le != hipSuccess) {
            err = fail(BWG_EDEVICE, "graph launch: %s", hipGetErrorString(le));
            break;
        }
        note_budgets(b, t_end.data(), kmin, kmax);
        for (auto *e : b->ens) note_ran(e, 0);
        for (size_t k = 0; k < n; ++k) t_end[k] = b->ens[k]->t_now + dt;
    }
    // the executable graph may still be running: destroy after the stream drains
    (void)hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    return err;
}
