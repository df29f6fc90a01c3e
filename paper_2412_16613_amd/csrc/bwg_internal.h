// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bwg {

// Random-stream domains of the draw contract (counter word 1, bits 24..31).
enum : uint32_t {
    DOM_EVENT = 1,
    DOM_BUDGET = 2,
    DOM_INIT = 3,
    DOM_PLAIN = 4,
    DOM_COMPONENT = 5,
    DOM_SHARED = 6,
};

// A dispatch covers fewer than 2^32 work-items (the dispatch packet counts
// them in 32 bits), so a launch with one work-item per replica (up to
// 2^32 - 1 of them, three per replica for plain-count copies) goes out in
// pieces of kLaunchSpan items, each kernel taking the first index of its
// piece.  Launches over words (at most 2^27) and lattice launches (whose
// schedule memory bounds the replicas far below 2^32) fit in one dispatch.
constexpr uint64_t kLaunchSpan = 1ull << 31;

#ifndef __HIPCC_RTC__   // host launch code: not part of the run-time compiled kernels
// f(i0, grid) once per piece [i0, i0 + span) of [0, n), span the largest
// multiple of block within kLaunchSpan (so a piece's last workgroup ends
// where the next piece starts, for any block size); nothing for n = 0.
template <class F>
inline hipError_t launch_pieces(uint64_t n, uint32_t block, F &&f)
{
    const uint64_t span = kLaunchSpan / block * block;
    for (uint64_t i0 = 0; i0 < n; i0 += span) {
        const uint64_t len = n - i0 < span ? n - i0 : span;
        f(i0, dim3((uint32_t)((len + block - 1) / block)));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
#endif

// Frank-family structure recognised for the bit-sliced kernel: the reaction
// table, after dropping trailing ghost reactions, is a subsequence of
//   A -> L, A -> D, A + L -> 2L, A + D -> 2D, L + D -> 2A
// with weights (cu, cu, 2^fa, 2^fa, 2^fi).  Absent reactions weigh 0.
struct FrankShape {
    uint32_t cu;     // weight constant of A -> L and of A -> D (0: absent)
    int32_t fa;      // log2 weight of the two autocatalytic reactions, -1 absent
    int32_t fi;      // log2 weight of L + D -> 2A, -1 absent
};

// Plain (one replica per thread) engine: 3 species, order <= 2, any table.
struct PlainReaction {
    int32_t kind;    // 0: unimolecular N_x; 1: N_x N_y; 2: N_x (N_x - 1) / 2
    int32_t x, y;    // reactant species
    int32_t d[3];    // state change
    uint32_t c;      // weight constant
};

struct WmArgs {
    uint32_t *planes;       // [3][nb_mem][wp] words, species (L, D, A)
    uint64_t *E;            // [32 wp] events done per replica
    uint64_t *Etgt;         // [32 wp] events to reach in this advance
    uint64_t *real;         // [wp] real events per 32-lane group
    uint64_t wp;            // padded words (row stride)
    uint64_t n_words;       // ceil(M / 32)
    uint64_t M;             // replicas
    uint64_t seed;
    uint64_t max_events;    // events per launch per word (0: no limit)
    uint32_t net_id;
    int32_t B;              // threshold planes (runtime, <= BC)
    uint32_t cu;
    int32_t fa, fi;
    int32_t nb_mem;         // count planes per species in memory (<= NB)
    uint32_t zs;            // shared threshold on [0, zs) for every replica (0: per replica)
    const uint32_t *ztab;   // shared thresholds of events [zbase, zbase + zlen)
    uint64_t zbase, zlen;
};

struct PlainArgs {
    int32_t *counts;        // [mp][3]
    uint64_t *E;
    uint64_t *Etgt;
    uint64_t *real;         // [mp] real events per replica
    uint64_t M;
    uint64_t seed;
    uint64_t max_events;
    uint32_t net_id;
    int32_t B;
    int32_t R;
    PlainReaction rx[16];
};

// Launchers (defined in the .hip files).  Each returns a hipError_t.
// block: threads per block (0: default); word_bits: replicas per thread (32,
// or 16 / 64 for the compile-time variants)
using WmLaunch = hipError_t (*)(const WmArgs &, hipStream_t, int block, int word_bits);
// Table of bit-sliced kernel instantiations: species planes NB, threshold
// plane capacity BC, product shift FA and unimolecular weight CU (-1: taken
// at run time).
// Initial counts of up to BWG_MAX_SPECIES species, passed by value.
struct SpeciesCounts {
    int32_t v[8];
};

struct WmVariant {
    int nb, bc, fa, cu;
    int nt, bs;  // molecule count and selection planes it is fixed to (nt = 0: any)
    WmLaunch fn;
};
extern const WmVariant kWmVariants[];
extern const int kWmVariantCount;

// Any 3-species network of order <= 2 on the bit-sliced state (reactions in
// table order).  Each reaction's weight is c_j h_j with h_j one of nine
// kinds: N_X (kind X), the pair counts N_L N_D, N_L N_A, N_D N_A (kinds 3,
// 4, 5) and N_X (N_X - 1) / 2 (kind 6 + X); d holds the state change.
constexpr int kGenMaxR = 16;
struct GenNet {
    int32_t R;
    uint32_t used;            // bit k: some reaction has kind k
    uint32_t change;          // bit j: reaction j changes the state
    int32_t n_slots;          // LDS slots, one per used kind
    uint32_t c[kGenMaxR];
    uint8_t kind[kGenMaxR];
    uint8_t slot[9];          // LDS slot of each used kind
    int8_t d[kGenMaxR][3];
};
using GenLaunch = hipError_t (*)(const WmArgs &, const GenNet &, hipStream_t);
struct GenVariant {
    int nb, bc;
    GenLaunch fn;
};
extern const GenVariant kGenVariants[];
extern const int kGenVariantCount;

hipError_t launch_plain(const PlainArgs &a, hipStream_t s, int block);
hipError_t launch_wm_lanes(const WmArgs &a, hipStream_t s);
// Shared thresholds of events [e0, e0 + len) into tab (len uint32).
hipError_t launch_shared_fill(uint32_t *tab, uint64_t e0, uint64_t len, uint64_t seed,
                              uint32_t net_id, uint32_t Z, hipStream_t s);

// ---- batches ----
struct BatchEns {
    WmArgs a;
    int32_t variant;        // persistent-kernel plane bucket
    int32_t pad;
};
struct BatchItem {
    uint32_t ens;           // index into the BatchEns array, | BATCH_ITEM_LANES
    uint32_t word0;         // first of 64 words (2 words for a lanes item)
};
constexpr uint32_t BATCH_ITEM_LANES = 0x80000000u;
struct BatchBudget {
    const uint64_t *T;      // Poisson table on the device (len 0: no events)
    uint64_t len;
    int64_t k_lo;
    uint64_t seed;
    uint64_t offset;        // first global replica of this ensemble
    uint64_t *adv;          // advance index (device)
    const uint64_t *E;
    uint64_t *Et;
    uint32_t net_id;
    uint32_t pad;
};
struct PersistVariant {
    int id, nb, bc;
};
extern const PersistVariant kPersistVariants[];
extern const int kPersistVariantCount;

hipError_t launch_persistent(const BatchEns *ens, const BatchItem *items, uint32_t n_items,
                             uint32_t *counter, int waves, uint64_t max_events, bool lanes,
                             hipStream_t s);
hipError_t launch_batch_budget(const BatchBudget *bb, int n_ens, uint64_t total, hipStream_t s);
hipError_t launch_batch_prologue(uint32_t *counter, hipStream_t s);
hipError_t launch_batch_epilogue(const BatchBudget *bb, int n_ens, hipStream_t s);

// ---- lattices ----
// Component schedule geometry: a group of LAT_GROUP_WORDS words (2048
// replicas) shares one component sequence; it is cut into chunks of LAT_CH
// events, each sorted into at most LAT_CH layers; a pass schedules and runs
// up to LAT_NCB chunks.
constexpr int LAT_GROUP_WORDS = 64;
constexpr int LAT_CH = 8192;
constexpr int LAT_NCB = 32;
constexpr int LAT_SLOT = 3 * LAT_CH + 64;   // uint32 per (group, chunk) slot
constexpr int LAT_MAX_SITES = 4096;

struct LatShape {
    int32_t lx, ly, S, P;
    int32_t B_r;            // threshold planes of a reaction component
    int32_t wx;             // planes of cu * A (A <= 2^P - 1)
    uint64_t cu;            // weight of A -> L and of A -> D
    uint64_t ca;            // weight of A + L -> 2L and of A + D -> 2D
    uint64_t ci;            // weight of L + D -> 2A
    uint64_t W_R;           // reaction component weight 2^B_r
    uint64_t W_H;           // hop component weight (T + 1) c_hop
    uint64_t Wsite;         // W_R + 4 W_H
    uint64_t C;             // S Wsite
    uint64_t thresh;        // 2^64 mod C
};

struct LatArgs {
    uint32_t *planes;       // [groups][S][64 words][3][P]
    const uint64_t *E;      // [32 words] events done before this advance
    const uint64_t *Et;     // [32 words] events to reach
    uint64_t *real;         // [words] real events (moves and reactions)
    uint64_t *blocked;      // [words] hops into full sites
    uint32_t *sched;        // [groups][LAT_NCB][LAT_SLOT]
    uint64_t M;
    uint64_t seed;
    uint64_t base;          // first event of chunk 0 of the advance
    uint32_t chunk0;        // first chunk of this pass
    uint32_t n_chunks;      // chunks in this pass (<= LAT_NCB)
    uint32_t net_id;
    uint32_t g0;            // event kernel: first group of the band
    uint32_t ng;            // event kernel: groups in the band
    uint32_t pad;
    LatShape sh;
};

using LatLaunch = hipError_t (*)(const LatArgs &, uint64_t words, hipStream_t);
// Event-kernel instantiations: species planes P, threshold-plane capacity
// bc, the weights cu, ca, ci (-1: taken at run time) and the words per
// workgroup slice ws.
struct LatVariant {
    int P, bc;
    int64_t cu, ca, ci;
    int ws, block;
    int stage;  // sites whose planes the launch keeps in LDS (0: none)
    LatLaunch fn;
};
extern const LatVariant kLatVariants[];
extern const int kLatVariantCount;

hipError_t launch_lat_init(uint32_t *planes, uint64_t words, uint64_t M, int S, int P, int mode,
                           const int32_t *sites_dev, const int32_t c3[3], int32_t lo, int32_t hi,
                           uint64_t seed, uint32_t net_id, uint64_t *E, uint64_t *Et,
                           uint64_t *real, uint64_t *blocked, hipStream_t s);
hipError_t launch_lat_schedule(const LatArgs &a, uint32_t n_groups, hipStream_t s);
hipError_t launch_lat_totals(const uint32_t *planes, uint64_t M, int S, int P, int32_t *dst,
                             hipStream_t s);
hipError_t launch_lat_sites(const uint32_t *planes, int S, int P, uint64_t first, uint64_t count,
                            int32_t *dst, hipStream_t s);
hipError_t launch_lat_histogram(const int32_t *tot, uint64_t M, int n_bins, uint64_t *dst,
                                hipStream_t s);

hipError_t launch_init_fixed(uint32_t *planes, int S, int nb, uint64_t wp, uint64_t M,
                             const int32_t *c, uint64_t *E, uint64_t *Et, uint64_t *real,
                             hipStream_t s);
hipError_t launch_init_multinomial(uint32_t *planes, int nb, uint64_t wp, uint64_t M,
                                   int64_t n_tot, uint64_t seed, uint32_t net_id,
                                   uint64_t *E, uint64_t *Etgt, uint64_t *real,
                                   hipStream_t s);
hipError_t launch_plain_init(int32_t *counts, uint64_t M, int mode, const int32_t c3[3],
                             int64_t n_tot, uint64_t seed, uint32_t net_id,
                             uint64_t *E, uint64_t *Etgt, uint64_t *real, hipStream_t s);
hipError_t launch_budget(const uint64_t *table, uint64_t len, int64_t k_lo,
                         uint64_t fixed_k, int use_table, uint64_t seed,
                         uint32_t net_id, const uint64_t *advance_dev, uint64_t M,
                         const uint64_t *E, uint64_t *Etgt, hipStream_t s);
hipError_t launch_add_u64(uint64_t *p, uint64_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_read_counts_planes(const uint32_t *planes, int S, int nb, uint64_t wp,
                                     uint64_t M, int32_t *dst, hipStream_t s);
hipError_t launch_read_counts_plain(const int32_t *counts, uint64_t M, int32_t *dst,
                                    hipStream_t s);
hipError_t launch_histogram(const uint32_t *planes, const int32_t *counts, int nb,
                            uint64_t wp, uint64_t M, int64_t n_tot, int n_bins,
                            uint64_t *dst, hipStream_t s);
hipError_t launch_gather_counts(const uint32_t *planes, const int32_t *counts, int nb,
                                uint64_t wp, uint64_t M, const uint32_t *sel, uint32_t n_sel,
                                int32_t *dst, hipStream_t s);
hipError_t launch_first_passage(const uint32_t *planes, const int32_t *counts, int nb,
                                uint64_t wp, uint64_t M, int32_t threshold, uint32_t k,
                                uint32_t *first, hipStream_t s);
hipError_t launch_copy_u64(const uint64_t *src, uint64_t *dst, uint64_t n, hipStream_t s);
hipError_t launch_sum_u64(const uint64_t *src, uint64_t n, uint64_t *dst2, int slot,
                          hipStream_t s);

}  // namespace bwg
