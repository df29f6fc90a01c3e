// Host-side structures shared by the C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "bwg.h"
#include "bwg_internal.h"

namespace bwg {

int fail(int code, const char *fmt, ...);

// A roctx range over a library call: a named range in rocprofv3's marker
// trace (--marker-trace), a function call otherwise.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::bwg::fail(BWG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// A bit-sliced kernel compiled at run time for one network (jit_host.cpp).
struct JitKernel;
void jit_release(JitKernel *k);
hipError_t jit_launch(const JitKernel *k, const WmArgs &a, hipStream_t s);

}  // namespace bwg

// Threshold planes the compiled bit-sliced kernels take (the precompiled
// ones and the lanes engine: 32).
constexpr int kMaxThresholdPlanes = 48;

struct Table {  // Poisson table of one mean
    int64_t k_lo;
    uint64_t len;
    std::vector<uint64_t> vals;  // the entries, for host-side draws
    uint64_t *host;              // pinned copy for uploads (made on first need);
                                 // lives as long as the network
};

struct bwg_net {
    int S = 0, R = 0;
    std::vector<int32_t> reac, prod;
    std::vector<double> rates;
    int64_t n_tot = 0;
    int32_t lx = 0, ly = 0;
    bwg_qnet q{};
    bwg::FrankShape shape{};
    bool shape_ok = false;
    bwg::PlainReaction prx[16]{};
    bool plain_ok = false;
    bwg::GenNet gen{};      // reaction table of the general bit-sliced kernel
    bool gen_ok = false;
    // open networks (BWG_OPEN: counts capped at n_tot, not conserved) and
    // networks of other than 3 species run only kernels compiled for them
    bool open = false;
    bool wide = false;      // S != 3 or open
    bool wide_ok = false;   // such a network fits the compiled general kernel
    // lattice networks
    bool lat = false;
    bwg::LatShape lsh{};
    int64_t c_lat[5]{};         // weights of the five Frank reactions
    int64_t c_hop = 0;
    int32_t T = 0;              // site capacity 2^P - 1
    bool lat_gpu = false;       // the event kernel implements this table
    std::mutex mu;
    std::map<uint64_t, Table> tables;  // keyed by the bits of mu
    bwg::JitKernel *jit = nullptr;     // compiled on the first ensemble that needs it
    bwg::JitKernel *jit_frank = nullptr;  // compiled Frank-family kernel (run-time weights)
    std::vector<char> jit_code, jit_frank_code;  // their code objects (gfx950)
    ~bwg_net()
    {
        for (auto &kv : tables)
            if (kv.second.host) (void)hipHostFree(kv.second.host);
        bwg::jit_release(jit);
        bwg::jit_release(jit_frank);
    }
};

struct bwg_ens {
    bwg_net *net = nullptr;
    uint64_t M = 0, seed = 0;
    uint32_t net_id = 0;
    int engine = 0, block = 0;
    int word_bits = 32;   // replicas per thread of the bit-sliced engine
    uint64_t table_cap = 0, epl = 0;
    uint8_t *buf = nullptr;
    uint64_t bytes = 0;
    uint64_t wp = 0;
    int nb = 0;
    const bwg::WmVariant *var = nullptr;
    const bwg::GenVariant *gvar = nullptr;  // general kernel (non-Frank or forced)
    const bwg::JitKernel *jit = nullptr;    // its per-network compiled form, if used
    const bwg::JitKernel *jit_frank = nullptr;  // compiled Frank kernel for a run-time variant
    bool want_jit_frank = false;                // build it at the first bit-sliced launch
    uint32_t *planes = nullptr;
    int32_t *counts = nullptr;
    uint64_t *E = nullptr, *Et = nullptr, *real = nullptr, *table = nullptr, *scratch = nullptr;
    uint64_t *adv_dev = nullptr;  // advance index on the device (scratch slot 8)
    double t_now = 0;
    uint64_t adv = 0;
    uint64_t lag = 0;      // bound on how far a word's lanes can be apart
    uint64_t pending = 0;  // bound on the events any word still has to run
    bool inited = false;
    uint64_t lanes_words = 0;  // in batches: trailing words run as lanes items
    uint32_t zs = 0;           // shared-threshold range (0: a threshold per replica)
    uint64_t zE = 0;           // with zs: the event every replica has reached
    uint64_t zbase = 0, zlen = 0;  // with zs: events whose thresholds the table holds
    // lattice ensembles
    bool lat = false;
    const bwg::LatVariant *lvar = nullptr;
    uint64_t words = 0, groups = 0;
    uint32_t *sched = nullptr;
    uint64_t *blocked = nullptr;
    int32_t *tot = nullptr;          // [32 words][3] species totals
    int32_t *sites_dev = nullptr;    // [S][3] staging of an initial lattice
    uint64_t emin = 0, emax = 0;     // bounds on min_i E_i and max_i E_i
    uint64_t base = 0, n_chunks = 0, cursor = 0;  // chunk window of the advance
    // event-kernel timing (BWG_OPT_TIME_KERNELS)
    bool timed = false;
    bool lat_stage = true;                      // lattices: LDS-staged event kernel
    std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;  // recorded, not yet read
    std::vector<hipEvent_t> spare;
    ~bwg_ens()
    {
        for (auto &m : marks) {
            (void)hipEventDestroy(m.first);
            (void)hipEventDestroy(m.second);
        }
        for (auto ev : spare) (void)hipEventDestroy(ev);
    }
};


namespace bwg {
// Bind a fresh ensemble e to dev_buf (validated: aligned, at least the state
// bytes of M replicas under o); what bwg_ensemble_create does after its
// checks, without allocating e.
int ens_bind(bwg_ens *e, const bwg_net *n, uint64_t M, uint64_t seed, uint32_t net_id,
             void *dev_buf, uint64_t buf_bytes, const bwg_opts *o);
// Cached Poisson table for mean mu (lives as long as the network); with
// pinned, also its pinned copy for uploads to the device.
int get_table(bwg_net *n, double mu, const Table **out, bool pinned = true);
// The network's run-time compiled kernel (compiled on the first call).
int jit_get(bwg_net *n, const JitKernel **out);
// The network's compiled Frank-family kernel (compiled on the first call),
// and whether the network fits that kernel's template parameters.
int jit_frank_get(bwg_net *n, const JitKernel **out);
bool jit_frank_fits(const bwg_net *n);
// Build, on the host only, the code objects of the general and/or the Frank
// kernel that are not built yet (later loads reuse them).
int jit_build_codes(bwg_net *n, bool general, bool frank);
// Budgets of one advance to t_end (no event launches); *kmin/*kmax bound K.
int schedule_ensemble(bwg_ens *e, double t_end, hipStream_t s, uint64_t *kmin, uint64_t *kmax);
// Bookkeeping after budgets with K in [kmin, kmax] were drawn.
void note_scheduled(bwg_ens *e, uint64_t kmin, uint64_t kmax);
// Bookkeeping after a pass that ran up to max_events per word (0: all).
void note_ran(bwg_ens *e, uint64_t max_events);

// Event-kernel timing: bracket one launch with HIP events when the ensemble
// was created with BWG_OPT_TIME_KERNELS (no-ops otherwise).
int mark_begin(bwg_ens *e, hipStream_t s, hipEvent_t *ev);
int mark_end(bwg_ens *e, hipStream_t s, hipEvent_t ev);

// Lattice networks and ensembles (lattice_host.cpp).
int lat_net_setup(bwg_net *n, const bwg_net_desc *d);
int lat_state_bytes(const bwg_net *n, uint64_t M, uint64_t table_cap, uint64_t *bytes);
int lat_bind(bwg_ens *e);
int lat_init(bwg_ens *e, int32_t mode, const int32_t *counts, hipStream_t s);
int lat_schedule(bwg_ens *e, double t_end, hipStream_t s);
int lat_step_schedule(bwg_ens *e, uint64_t n_events, hipStream_t s);
int lat_run(bwg_ens *e, uint64_t max_events, hipStream_t s);
int lat_read_counts(bwg_ens *e, int32_t *dst, hipStream_t s);
int lat_histogram(bwg_ens *e, int32_t n_bins, uint64_t *dst, hipStream_t s);
}
