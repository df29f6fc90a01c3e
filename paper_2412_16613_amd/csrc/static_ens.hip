// Allocation-free fixed-K run of a well-mixed ensemble: the whole device
// state of the ensemble (bit planes, per-replica event counters, per-word
// real-event counters, the advance index) lives in one file-scope device
// array instead of a caller buffer, so a caller that cannot allocate device
// memory (code under HIP graph capture, a serving loop that forbids it) can
// still run the bit-parallel step.  The kernels are the ones
// bwg_ensemble_step launches; they receive this array's device address as
// they receive the caller's buffer there.

#include <hip/hip_runtime.h>

#include <mutex>

#include "host_internal.h"

namespace {

// Device-side home of the ensemble state, one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device memory: only its address from hipGetSymbolAddress is used.
static __device__ __align__(256) uint8_t scratch[BWG_STATIC_STATE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// The array's device address on the current device (looked up once per
// device, with that device current).
int scratch_address(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return bwg::fail(BWG_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (rc != hipSuccess || !p)
            return bwg::fail(BWG_EDEVICE, "hipGetSymbolAddress(scratch): %s",
                             hipGetErrorString(rc));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BWG_OK;
}

}  // namespace

extern "C" int bwg_ensemble_step_static(const bwg_net *n, uint64_t n_replicas, uint64_t seed,
                                        uint32_t net_id, const int32_t *counts, uint64_t n_events,
                                        int32_t *dev_counts, void *stream)
{
    if (!n || !counts || !dev_counts) return bwg::fail(BWG_EINVAL, "null argument");
    if (n->lat) return bwg::fail(BWG_EUNSUPPORTED, "the static-state run is for well-mixed networks");
    bwg_opts o{};
    o.engine = BWG_ENGINE_BITWISE;
    o.flags = BWG_OPT_NO_JIT;  // a run-time compile would load code (allocate)
    uint64_t need = 0;
    int rc = bwg_ensemble_state_bytes(n, n_replicas, &o, &need);
    if (rc) return rc;
    if (need > BWG_STATIC_STATE_BYTES)
        return bwg::fail(BWG_ERANGE,
                         "%llu replicas need %llu bytes of state, beyond the %llu of the static "
                         "array",
                         (unsigned long long)n_replicas, (unsigned long long)need,
                         (unsigned long long)BWG_STATIC_STATE_BYTES);
    void *buf = nullptr;
    rc = scratch_address(&buf);
    if (rc) return rc;
    // the ensemble handle lives on this stack frame; init rewrites every
    // state word the step reads, so nothing depends on the last call's
    // contents of the array
    bwg_ens e;
    rc = bwg::ens_bind(&e, n, n_replicas, seed, net_id, buf, BWG_STATIC_STATE_BYTES, &o);
    if (rc) return rc;
    rc = bwg_ensemble_init(&e, BWG_INIT_FIXED, counts, stream);
    if (rc) return rc;
    rc = bwg_ensemble_step(&e, n_events, stream);
    if (rc) return rc;
    return bwg_ensemble_read_counts(&e, dev_counts, stream);
}
