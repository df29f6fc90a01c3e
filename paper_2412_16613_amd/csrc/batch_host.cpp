// C ABI of batches: many ensembles advanced by one persistent launch, and a
// graph of one batch advance replayed for repeated equal time steps.

#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "host_internal.h"

using namespace bwg;

struct bwg_batch {
    std::vector<bwg_ens *> ens;
    std::vector<int> bucket;       // persistent-kernel plane bucket per ensemble
    std::vector<double> cost;      // VALU cost of one event of a word, per ensemble
    int waves = 0;
    int order = 0;
    uint64_t max_items = 0;
    // device layout (caller buffer)
    BatchEns *d_ens = nullptr;
    BatchBudget *d_budget = nullptr;
    BatchItem *d_items = nullptr;
    uint32_t *d_counter = nullptr;
    // pinned staging and the event that guards its reuse
    BatchBudget *h_budget = nullptr;
    BatchItem *h_items = nullptr;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    ~bwg_batch()
    {
        if (staged_pending) (void)hipEventSynchronize(staged);
        if (staged) (void)hipEventDestroy(staged);
        if (h_budget) (void)hipHostFree(h_budget);
        if (h_items) (void)hipHostFree(h_items);
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

static uint64_t n_items_of(const bwg_ens *e) { return (((e->M + 31) / 32) + 63) / 64; }

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

static uint64_t total_bytes(int n, uint64_t items)
{
    uint64_t a, b, c, d;
    return layout_bytes(n, items, &a, &b, &c, &d);
}

static int check_members(bwg_ens *const *ens, int32_t n, uint64_t *items)
{
    if (!ens || n < 1) return fail(BWG_EINVAL, "empty batch");
    uint64_t it = 0;
    for (int k = 0; k < n; ++k) {
        const bwg_ens *e = ens[k];
        if (!e) return fail(BWG_EINVAL, "null ensemble %d", k);
        if (e->engine != BWG_ENGINE_BITWISE)
            return fail(BWG_EUNSUPPORTED, "ensemble %d: batches run the bit-sliced engine", k);
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
    *bytes = total_bytes(n, items);
    return BWG_OK;
}

extern "C" int bwg_batch_create(bwg_ens *const *ens, int32_t n, void *dev_buf, uint64_t buf_bytes,
                                const bwg_batch_opts *opts, void *stream, bwg_batch **out)
{
    if (!out || !dev_buf) return fail(BWG_EINVAL, "null argument");
    *out = nullptr;
    if ((uintptr_t)dev_buf & 255) return fail(BWG_EINVAL, "device buffer not 256-byte aligned");
    uint64_t items;
    int rc = check_members(ens, n, &items);
    if (rc) return rc;
    const uint64_t need = total_bytes(n, items);
    if (buf_bytes < need)
        return fail(BWG_ENOMEM, "batch buffer of %llu bytes, need %llu",
                    (unsigned long long)buf_bytes, (unsigned long long)need);
    auto b = new bwg_batch();
    b->ens.assign(ens, ens + n);
    b->waves = (opts && opts->waves > 0) ? opts->waves : 2048;
    b->order = opts ? opts->order : 0;
    b->max_items = items;
    uint64_t o_ens, o_bud, o_it, o_cnt;
    layout_bytes(n, items, &o_ens, &o_bud, &o_it, &o_cnt);
    uint8_t *base = (uint8_t *)dev_buf;
    b->d_ens = (BatchEns *)(base + o_ens);
    b->d_budget = (BatchBudget *)(base + o_bud);
    b->d_items = (BatchItem *)(base + o_it);
    b->d_counter = (uint32_t *)(base + o_cnt);
    hipStream_t s = (hipStream_t)stream;
    int err = BWG_OK;
    do {
        if (hipHostMalloc((void **)&b->h_budget, sizeof(BatchBudget) * n, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&b->h_items, sizeof(BatchItem) * items, hipHostMallocDefault) !=
                hipSuccess ||
            hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
            err = fail(BWG_EDEVICE, "pinned staging allocation failed");
            break;
        }
        std::vector<BatchEns> he(n);
        for (int k = 0; k < n; ++k) {
            const bwg_ens *e = ens[k];
            const bwg_net *nt = e->net;
            const int bk = pick_bucket(e);
            b->bucket.push_back(bk);
            const PersistVariant &v = kPersistVariants[bk];
            // per-event issue cost of the bucket: RNG quads + planes (an estimate
            // used only to order the queue)
            b->cost.push_back(100.0 * ((nt->q.B + 3) / 4) + 8.0 * v.bc + 40.0 * v.nb);
            WmArgs &a = he[k].a;
            memset(&a, 0, sizeof a);
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
            he[k].variant = bk;
            he[k].pad = 0;
        }
        if (hipMemcpyAsync(b->d_ens, he.data(), sizeof(BatchEns) * n, hipMemcpyHostToDevice, s) !=
            hipSuccess) {
            err = fail(BWG_EDEVICE, "upload of batch descriptors failed");
            break;
        }
        if (hipStreamSynchronize(s) != hipSuccess) {
            err = fail(BWG_EDEVICE, "stream synchronisation failed");
            break;
        }
    } while (0);
    if (err) {
        delete b;
        return err;
    }
    *out = b;
    return BWG_OK;
}

extern "C" void bwg_batch_destroy(bwg_batch *b) { delete b; }

// Stage tables, budgets and the ordered queue of one advance to t_end[k].
static int stage(bwg_batch *b, const double *t_end, hipStream_t s, double *mu_out)
{
    const int n = (int)b->ens.size();
    if (b->staged_pending) {
        HIP_TRY(hipEventSynchronize(b->staged));
        b->staged_pending = false;
    }
    uint64_t offset = 0;
    std::vector<std::pair<double, BatchItem>> q;
    q.reserve(b->max_items);
    for (int k = 0; k < n; ++k) {
        bwg_ens *e = b->ens[k];
        if (!e->inited) return fail(BWG_EINVAL, "ensemble %d not initialised", k);
        if (!(t_end[k] >= e->t_now))
            return fail(BWG_EINVAL, "ensemble %d: t_end %g before t_now %g", k, t_end[k], e->t_now);
        const double mu = e->net->q.lambda * (t_end[k] - e->t_now);
        mu_out[k] = mu;
        BatchBudget &bb = b->h_budget[k];
        memset(&bb, 0, sizeof bb);
        uint64_t kmax = 0, kmin = 0;
        if (mu > 0) {
            const Table *t;
            int rc = get_table(e->net, mu, &t);
            if (rc) return rc;
            if (t->len > e->table_cap)
                return fail(BWG_ERANGE, "ensemble %d: Poisson table of %llu entries exceeds %llu",
                            k, (unsigned long long)t->len, (unsigned long long)e->table_cap);
            HIP_TRY(hipMemcpyAsync(e->table, t->host, t->len * 8, hipMemcpyHostToDevice, s));
            bb.T = e->table;
            bb.len = t->len;
            bb.k_lo = t->k_lo;
            kmin = (uint64_t)t->k_lo;
            kmax = (uint64_t)t->k_lo + t->len;
        }
        bb.seed = e->seed;
        bb.offset = offset;
        bb.adv = e->adv_dev;
        bb.E = e->E;
        bb.Et = e->Et;
        bb.net_id = e->net_id;
        offset += e->M;
        const double c = b->cost[k] * (double)(kmax + e->lag);
        const uint64_t words = (e->M + 31) / 32;
        for (uint64_t w0 = 0; w0 < words; w0 += 64)
            q.push_back({c, BatchItem{(uint32_t)k, (uint32_t)w0}});
        (void)kmin;
    }
    if (b->order == 0)
        std::stable_sort(q.begin(), q.end(),
                         [](const std::pair<double, BatchItem> &x,
                            const std::pair<double, BatchItem> &y) { return x.first > y.first; });
    for (size_t i = 0; i < q.size(); ++i) b->h_items[i] = q[i].second;
    HIP_TRY(hipMemcpyAsync(b->d_budget, b->h_budget, sizeof(BatchBudget) * n,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->d_items, b->h_items, sizeof(BatchItem) * q.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(b->staged, s));
    b->staged_pending = true;
    return BWG_OK;
}

// The kernels of one batch advance (budgets, advance indices, queue reset,
// persistent event kernel); all graph-capturable.
static int enqueue(bwg_batch *b, uint64_t total_replicas, hipStream_t s)
{
    const int n = (int)b->ens.size();
    HIP_TRY(launch_batch_budget(b->d_budget, n, total_replicas, s));
    HIP_TRY(launch_batch_epilogue(b->d_budget, n, s));
    HIP_TRY(launch_batch_prologue(b->d_counter, s));
    HIP_TRY(launch_persistent(b->d_ens, b->d_items, (uint32_t)b->max_items, b->d_counter, b->waves,
                              s));
    return BWG_OK;
}

static void finish_host(bwg_batch *b, const double *t_end, const double *mu)
{
    for (size_t k = 0; k < b->ens.size(); ++k) {
        bwg_ens *e = b->ens[k];
        const Table *t = nullptr;
        if (mu[k] > 0 && get_table(e->net, mu[k], &t) == BWG_OK) e->lag += t->len;
        e->t_now = t_end[k];
        e->adv += 1;
    }
}

extern "C" int bwg_batch_advance(bwg_batch *b, const double *t_end, void *stream)
{
    if (!b || !t_end) return fail(BWG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> mu(b->ens.size());
    int rc = stage(b, t_end, s, mu.data());
    if (rc) return rc;
    uint64_t total = 0;
    for (auto *e : b->ens) total += e->M;
    rc = enqueue(b, total, s);
    if (rc) return rc;
    finish_host(b, t_end, mu.data());
    return BWG_OK;
}

extern "C" int bwg_batch_graph_advance(bwg_batch *b, double dt, int32_t n_steps, void *stream)
{
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
    std::vector<double> t_end(n), mu(n);
    for (size_t k = 0; k < n; ++k) t_end[k] = b->ens[k]->t_now + dt;
    int rc = stage(b, t_end.data(), s, mu.data());
    if (rc) return rc;
    uint64_t total = 0;
    for (auto *e : b->ens) total += e->M;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = enqueue(b, total, s);
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
        finish_host(b, t_end.data(), mu.data());
        for (size_t k = 0; k < n; ++k) t_end[k] = b->ens[k]->t_now + dt;
    }
    // the executable graph may still be running: destroy after the stream drains
    (void)hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    return err;
}
