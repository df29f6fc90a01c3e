/*
 * bwg.h -- C ABI of the bit-parallel Gillespie library for MI355X (gfx950).
 *
 * The library simulates many independent replicas of a chemical reaction
 * network with Gillespie's exact stochastic simulation algorithm, holding the
 * species counts of 32 replicas bit-sliced in each 32-bit word (one replica
 * per bit lane, one word per bit of the count) and selecting and applying
 * reactions with word-wide logic and ripple-carry arithmetic.  This is the
 * bitwise Gillespie method of Castellana and Lacoste, "Parallelization of
 * Gillespie algorithm based on binary words" (Sec. 4 and App. B), with one
 * random threshold per replica instead of one shared by all copies.
 *
 * Conventions
 *   - Every function returns an int status: BWG_OK (0) or a negative code
 *     below; bwg_last_error() returns a thread-local message for the last
 *     failure on the calling thread.
 *   - Device memory is owned by the caller: an ensemble lives entirely in one
 *     caller-allocated device buffer of bwg_ensemble_state_bytes() bytes
 *     (256-byte aligned).  Output buffers are caller-owned device pointers.
 *   - Streams are passed as `void*` holding a hipStream_t (NULL = the null
 *     stream).  Calls marked "async" only enqueue work on that stream;
 *     results are valid once the stream has synchronised.
 *   - Handles are not thread-safe; distinct handles may be used from
 *     distinct threads.  A network must outlive its ensembles.
 *   - Species order of the Frank model is (L, D, A): the two enantiomers and
 *     the achiral activator of Sec. 2 of the paper.
 */
#ifndef BWG_H
#define BWG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BWG_OK = 0,
    BWG_EINVAL = -1,       /* invalid argument or network                     */
    BWG_ERANGE = -2,       /* value outside what the planes/tables can hold  */
    BWG_ENOMEM = -3,       /* caller buffer too small                         */
    BWG_EDEVICE = -4,      /* HIP runtime error (message has the HIP text)    */
    BWG_EUNSUPPORTED = -5  /* valid network the GPU kernels do not implement  */
};

#define BWG_MAX_SPECIES 8
#define BWG_MAX_REACTIONS 16

/* flags of bwg_net_desc */
#define BWG_EXACT_INTEGER 1u   /* rates are the integer weights (paper mode) */
/* An open network: reactions need not conserve the molecule count (the
 * general networks the paper leaves to future work, Sec. 6).  Every species
 * count is capped at n_tot: a selected reaction whose firing would leave a
 * count above n_tot does nothing (a null event; the chain on the truncated
 * state space {0 <= N_x <= n_tot}).  Initial counts are each at most n_tot.
 * Runs on the bit-sliced engine's kernel compiled for the network only. */
#define BWG_OPEN 2u

/* engines of bwg_opts */
#define BWG_ENGINE_BITWISE 0   /* bit-sliced words, 32 replicas per lane: the
                                  Frank-family kernel (incremental products,
                                  App. B) for the five Frank reactions with or
                                  without ghosts, the general kernel for any
                                  other 3-species network of order <= 2      */
#define BWG_ENGINE_PLAIN 1     /* comparator: one replica per thread, int32   */
#define BWG_ENGINE_LANES 2     /* the bit-plane state and draws of BITWISE, one
                                  replica per thread: identical results, a
                                  shorter chain per event, more work per
                                  replica-event (Frank family only)          */

/* initial-state modes of bwg_ensemble_init */
#define BWG_INIT_FIXED 0        /* every replica starts from counts[0..S-1]   */
#define BWG_INIT_MULTINOMIAL 1  /* each molecule L, D, A w.p. 1/4, 1/4, 1/2   */
#define BWG_INIT_UNIFORM_SITE 2 /* lattice: A uniform in {counts[0]..counts[1]}
                                   on every site, L = D = 0                    */
#define BWG_INIT_SITES 3        /* lattice: every replica starts from the site
                                   counts counts[s*3 + x], s < lx*ly           */

typedef struct bwg_net bwg_net;
typedef struct bwg_ens bwg_ens;

/*
 * A reaction network.  Reaction j consumes reactants[j*S + x] molecules of
 * species x and produces products[j*S + x]; total order 1 or 2; every
 * reaction must conserve the molecule count (the paper's networks conserve
 * N_tot, Sec. 2) unless the network is open (BWG_OPEN).  rates[j] is the
 * mass-action constant: the propensity is rates[j] * h_j(N) with h_j = N_X,
 * N_X N_Y or N_X (N_X - 1)/2 (the forms of Eq. (7) of the paper).  Networks
 * of 3 species that conserve the count run every engine; other species
 * counts (1..BWG_MAX_SPECIES) and open networks run the bit-sliced kernel
 * compiled for the network, with changes of at most 2 per species and
 * reaction.  All pointers are read during the call only.
 */
typedef struct {
    int32_t n_species;          /* S, <= BWG_MAX_SPECIES                      */
    int32_t n_reactions;        /* R, <= BWG_MAX_REACTIONS                    */
    const int32_t *reactants;   /* [R][S]                                     */
    const int32_t *products;    /* [R][S]                                     */
    const double *rates;        /* [R], finite, >= 0                          */
    int64_t n_tot;              /* molecules per replica                      */
    int32_t lx, ly;             /* 0, 0: well-mixed                           */
    const double *hop_rates;    /* [S] per molecule per direction, or NULL    */
    int32_t site_planes;        /* bits per species count on a lattice site   */
    int32_t precision_bits;     /* rate quantisation, 0 = default (7)         */
    uint32_t flags;             /* BWG_EXACT_INTEGER, BWG_OPEN                */
    uint32_t reserved;
} bwg_net_desc;

/*
 * The integer form of a network (what the kernels run and the oracle checks):
 * reaction j has weight w_j(N) = c[j] * h_j(N); the weights are in units of
 * 1/s per unit time; W = 2^B bounds sum_j w_j(N) over every state with
 * N_tot molecules; the uniformised chain runs lambda = 2^B / s events per
 * replica per unit time, each event picking reaction j with probability
 * w_j / 2^B and nothing otherwise (the role of the ghost reactions, Eq. (9)).
 * b planes hold one species count (2^b > N_tot).
 */
typedef struct {
    int32_t n_species, n_reactions;
    int64_t c[BWG_MAX_REACTIONS];
    int32_t f;            /* scale exponent: s = 2^f / k_ref                  */
    int32_t B;            /* threshold planes                                 */
    int32_t b;            /* planes per species count                         */
    int32_t gpu_ok;       /* 1 if the GPU kernels implement this network      */
    double s;
    double lambda;
    int64_t max_total;    /* max_N sum_j w_j(N)                               */
    int64_t z_shared;     /* Z of BWG_OPT_SHARED_THRESHOLD: sum_j w_j(N) if it
                             is the same for every N (ghost reactions, Eq. (9)),
                             else 2^B; 0 if Z >= 2^32                          */
} bwg_qnet;

/*
 * Integer form of a lattice network (lx, ly > 0).  The paper's method is for
 * one well-mixed reactor; it names ensembles of small compartments as the
 * use it aims at (Sec. 1, Sec. 6) without giving their chain, so the library
 * defines it: every site is a Frank reactor (reactions in the order A -> L,
 * A -> D, A + L -> 2L, A + D -> 2D, L + D -> 2A, weights c_j h_j of the site
 * counts) whose molecules hop to each of the 4 periodic neighbours at weight
 * c_hop; a site holds at most T = 2^P - 1 molecules and a hop into a full
 * site does nothing.  Uniformisation by components: a reaction component per
 * site of weight 2^B_r (2^B_r >= max_site, the largest site weight sum) and
 * a hop component per (site, direction) of weight (T + 1) c_hop, C in all;
 * lambda = C / s events per replica per unit time.  Each event draws one
 * component shared by the 2048 replicas of a group, then per replica a
 * threshold (reaction) or a molecule index j in [0, T] (hop: A if j < n_A,
 * L if j < n_A + n_L, D if j < n_site).
 */
typedef struct {
    int32_t lx, ly, sites;      /* periodic lattice, sites = lx * ly          */
    int32_t P, T;               /* planes per species count, site capacity    */
    int32_t B_r;                /* threshold planes of a reaction component   */
    int64_t c_hop;              /* hop weight per molecule and direction      */
    uint64_t C;                 /* total component weight                     */
    int64_t max_site;           /* largest site weight sum                    */
    double s, lambda;           /* scale 2^f / k_ref; C / s                   */
} bwg_lattice_info;

/* flags of bwg_opts */
#define BWG_OPT_TIME_KERNELS 1u  /* record HIP events around every event-kernel
                                    launch (bwg_ensemble_kernel_time)         */
/* The paper's shared-threshold variant (Sec. 4, after the bitwise step; the
 * gain it measures in Sec. 5): at event e every replica compares the same n,
 * uniform on [0, z_shared), against its own cumulative weights, so one random
 * number serves all replicas; and an advance draws one event budget for all
 * of them (the paper's single time step per iteration, Eq. (12)), Poisson with
 * mean (z_shared / s) (t_end - t_now): events arrive at the paper's constant
 * total propensity instead of lambda.  The replicas stay exact marginal copies
 * of the chain but are no longer independent of each other, and they move in
 * lockstep.  Only for the bit-sliced and lanes engines on well-mixed networks
 * (EUNSUPPORTED otherwise; ERANGE when z_shared is 0); batches refuse such
 * ensembles (EUNSUPPORTED).  A step or advance runs in launches of at most
 * 2 * table_capacity events (and at most events_per_launch, if set), each
 * after a fill of its thresholds into the ensemble's table region. */
#define BWG_OPT_SHARED_THRESHOLD 2u
/* Run a Frank-family network on the general bit-sliced kernel, the one
 * every other 3-species network of order <= 2 takes on the bit-sliced engine:
 * weights c_j h_j recomputed from the planes at every event (h = N_X,
 * N_X N_Y or N_X (N_X - 1) / 2, Eq. (7)), first crossing in table order,
 * the same draws, so the same results as the Frank kernel at a higher cost
 * per event.  Bit-sliced engine on well-mixed networks only (EUNSUPPORTED
 * otherwise), not with BWG_OPT_SHARED_THRESHOLD. */
#define BWG_OPT_GENERIC_KERNEL 4u
/* Networks on the general path run, by default, a kernel compiled at run
 * time (hipRTC) for their own reaction table on the first ensemble created:
 * weight kinds in registers, one compile-time shifted subtraction per set bit
 * of each c_j, trailing reactions that change nothing left out; same results
 * as the precompiled general kernel.  Creation fails with EDEVICE (and the
 * compiler's log in bwg_last_error) if that compile fails.  Likewise a
 * Frank-family network whose product shift and unimolecular weight match no
 * precompiled variant runs the Frank kernels compiled for its plane counts
 * and weights; that compile happens at the ensemble's first bit-sliced
 * launch (default block size, per-replica or shared thresholds; batches
 * never run it),
 * which fails with EDEVICE if the compile fails, and gives the results of the
 * precompiled run-time weight kernels.  This flag keeps the precompiled
 * kernels instead. */
#define BWG_OPT_NO_JIT 8u
/* Lattices: run the event kernel that keeps every site's planes in memory.
 * By default ensembles of 512 words (16384 replicas) and more, on a lattice
 * with 4 planes per species and the weights of the precompiled lattice kernel,
 * run the kernel that keeps the planes of the first BWG_LAT_STAGE_SITES sites
 * of each word in LDS for the whole launch (copied in at the start and back at
 * the end); the results are the same either way.  Ignored for well-mixed
 * networks. */
#define BWG_OPT_NO_LDS_STAGE 16u
#define BWG_LAT_STAGE_SITES 840
/* Lattice schedule geometry: the component events of a group of 2048
 * replicas are cut into chunks of BWG_LAT_CHUNK_EVENTS, each sorted into
 * conflict-free layers; a pass schedules up to BWG_LAT_PASS_CHUNKS chunks of
 * every group and runs them.  The schedule takes BWG_LAT_PASS_CHUNKS x
 * (3 BWG_LAT_CHUNK_EVENTS + 64) x 4 bytes of the state per group. */
#define BWG_LAT_CHUNK_EVENTS 8192
#define BWG_LAT_PASS_CHUNKS 32

typedef struct {
    int32_t engine;              /* BWG_ENGINE_*                              */
    int32_t block;               /* threads per block of the event kernels:
                                    0 (default), 64, 128, 192 or 256 (EINVAL
                                    otherwise)                               */
    uint64_t table_capacity;     /* Poisson-table entries, 0 = default 65536  */
    uint64_t events_per_launch;  /* 0 = whole advance in one launch           */
    uint64_t flags;              /* BWG_OPT_*                                 */
    uint64_t word_bits;          /* replicas per thread of the bit-sliced
                                    engine: 0 or 32 (a 32-bit word), 16 (half
                                    a word) or 64 (two words); the draws are
                                    keyed by the 32-lane word and the lane, so
                                    results do not depend on it.  16 and 64
                                    run the one-wave-per-thread form on
                                    precompiled compile-time weights only (the
                                    named workloads, the paper's network):
                                    EUNSUPPORTED otherwise, EINVAL for other
                                    values.  The paper's words are 64-bit
                                    integers (Sec. 4, Sec. 5).               */
    uint64_t reserved[2];
} bwg_opts;

typedef struct {
    uint64_t n_replicas;
    uint64_t advance_index;      /* advances done since init                  */
    double t_now;
    uint64_t events_total;       /* sum over replicas of events run           */
    uint64_t real_total;         /* of which changed the state                */
} bwg_stats;

/* ---- networks (host only, synchronous) ------------------------------- */

/* Validate and quantise a network (integer weights c_j, scale, bound 2^B).
 * The bound: for 3 species conserving the count, the largest total weight
 * over the simplex (exactly: for each first count the total is an integer
 * quadratic in the second, whose extremes lie at the ends and next to the
 * vertex); else sum_j c_j max h_j, each reaction's
 * largest factor over the simplex of n_tot molecules (N_X: n_tot, pairs
 * floor(n/2) ceil(n/2), N_X (N_X - 1)/2: n(n-1)/2) or, open, over the box of
 * counts at most n_tot (n, n^2, n(n-1)/2).
 * EINVAL: order not in {1,2}, not count-conserving (and not open), negative
 * or non-finite rate, n_tot < 1, sizes out of range; ERANGE: weights beyond
 * 32 bits, a bound beyond 48 threshold planes, or n_tot beyond the count
 * planes.  Beyond 32 threshold planes (rates quantised at more bits of
 * precision, precision_bits) only the bit-sliced engine runs the network,
 * on the kernels compiled for it at run time (state_bytes refuses the other
 * engines, BWG_OPT_NO_JIT, explicit block sizes, other word widths and shared
 * thresholds; batches refuse such ensembles);
 * EUNSUPPORTED: a lattice that is open or not of 3 species.  The returned
 * handle is owned by the caller (bwg_net_destroy). */
int bwg_net_create(const bwg_net_desc *desc, bwg_net **out);
int bwg_net_quantized(const bwg_net *net, bwg_qnet *out);

/* The lattice form of a network created with lx, ly > 0 (EINVAL otherwise).
 * For such networks bwg_net_quantized reports c[0..4], f, s, B = B_r,
 * b = P, lambda and max_total = max_site.  Lattice networks need the five
 * Frank reactions in the order above, one hop rate for all species,
 * site_planes 1..8 and at most 4096 sites (EUNSUPPORTED / ERANGE). */
int bwg_net_lattice(const bwg_net *net, bwg_lattice_info *out);
void bwg_net_destroy(bwg_net *net);

/* Compile now, on the host and without touching a device, the kernels that
 * a bit-sliced ensemble of this network under default options would compile
 * at run time (hipRTC, gfx950): the general kernel for networks outside the
 * Frank family, open networks and other species counts (the general networks
 * Sec. 6 proposes, on the Sec. 4 state); the Frank-family
 * kernel with the network's weights as constants where no precompiled
 * variant has them.  Ensembles created later only load the code (done once
 * per network).  *built (may be NULL) gets BWG_JIT_GENERAL | BWG_JIT_FRANK
 * for the kernels this network uses, 0 when it runs precompiled kernels
 * only or is a lattice.  EUNSUPPORTED if no bit-sliced kernel runs the
 * network; EDEVICE with the compiler's log if a compile fails.  Thread-safe
 * per network. */
#define BWG_JIT_GENERAL 1u
#define BWG_JIT_FRANK 2u
int bwg_net_compile(bwg_net *net, uint32_t *built);

/* Poisson inverse-CDF table of the event budget for mean mu (host):
 * table[j] = floor(2^64 P(K <= k_lo + j)), j < len, ending at the first
 * entry equal to 2^64-1.  ERANGE if cap entries do not suffice (len then
 * holds the size needed). */
int bwg_poisson_table(double mu, int64_t *k_lo, uint64_t *table, uint64_t cap,
                      uint64_t *len);

/* ---- ensembles ---------------------------------------------------------- */

/* Device bytes an ensemble of n_replicas needs (opts may be NULL): the bit
 * planes of every species count (Sec. 4, Eqs. (15)-(19): plane q holds bit q
 * of the counts of 32 replicas, 32 * ceil(n_replicas / 32) lanes, words
 * padded to multiples of 64), the per-replica event counters and the Poisson
 * table region.  EINVAL for n_replicas = 0 or >= 2^32 or a bad block size;
 * EUNSUPPORTED when no kernel of the chosen engine runs the network. */
int bwg_ensemble_state_bytes(const bwg_net *net, uint64_t n_replicas,
                             const bwg_opts *opts, uint64_t *bytes);

/* Bind an ensemble of M copies of the network (the paper's M replicas of one
 * network sharing N_tot, Sec. 4) to a caller buffer (device, 256-byte
 * aligned, owned by the caller, which must outlive the ensemble).  seed and
 * net_id key every random draw (Philox4x32-10 counters); replicas of equal
 * (seed, net_id, index) see identical draws in any ensemble, batch or word
 * width.  No device work is enqueued.  ENOMEM if buf_bytes is below
 * bwg_ensemble_state_bytes; EINVAL for a null or misaligned buffer. */
int bwg_ensemble_create(const bwg_net *net, uint64_t n_replicas, uint64_t seed,
                        uint32_t net_id, void *dev_buf, uint64_t buf_bytes,
                        const bwg_opts *opts, bwg_ens **out);

/* Set every replica's initial state and reset time, event counters and the
 * advance index.  mode BWG_INIT_FIXED takes counts[S] (host pointer, summing
 * to n_tot; open networks: each at most n_tot, ERANGE otherwise);
 * BWG_INIT_MULTINOMIAL draws the paper's racemic multinomial start (Frank
 * species only).  Lattices take BWG_INIT_FIXED (counts[3] on every
 * site), BWG_INIT_SITES (counts[sites*3]) or BWG_INIT_UNIFORM_SITE (counts =
 * {lo, hi}; the draw of replica i, site s is exact: 32-bit multiply-shift
 * with rejection on INIT draws); ERANGE if a site would exceed T.  Async. */
int bwg_ensemble_init(bwg_ens *ens, int32_t mode, const int32_t *counts,
                      void *stream);

/* Advance every replica to time t_end >= t_now: each replica draws its event
 * count K ~ Poisson(lambda (t_end - t_now)) by inversion of one 64-bit
 * uniform, then runs K events of the uniformised chain (Sec. 3 update rule,
 * in the bitwise form of Sec. 4).  EINVAL if t_end < t_now; ERANGE if the
 * Poisson table exceeds the table capacity.  Async. */
int bwg_ensemble_advance(bwg_ens *ens, double t_end, void *stream);

/* The two halves of an advance, for callers that interleave the events of
 * many ensembles (continuous batching): bwg_ensemble_schedule draws every
 * replica's event budget for an advance to t_end (and moves t_now to t_end)
 * without running events; bwg_ensemble_run runs pending events, at most
 * max_events per word (0: all).  Splitting an advance this way, and running
 * it in any number of capped passes, gives the same result as
 * bwg_ensemble_advance.  Async. */
int bwg_ensemble_schedule(bwg_ens *ens, double t_end, void *stream);
int bwg_ensemble_run(bwg_ens *ens, uint64_t max_events, void *stream);
/* Lattices run whole chunks of 8192 events of their component sequence, so a
 * capped pass may run up to 8191 events beyond max_events; a lattice accepts
 * a new schedule, advance or step only once its pending bound is 0 (EINVAL
 * otherwise), and its per-replica event counts move to their targets when
 * the last chunk has run. */

/* Host-side upper bound on the events any word still has to run (0 once
 * every scheduled event has been launched).  No device work, no sync. */
int bwg_ensemble_pending(const bwg_ens *ens, uint64_t *bound);

/* Run exactly n_events more events in every replica, without time (the
 * paper's fixed number of iterations, Sec. 5).  Async. */
int bwg_ensemble_step(bwg_ens *ens, uint64_t n_events, void *stream);

/* Counts of every replica: dev_dst[i*S + x], int32, species order of the
 * network; on a lattice the species totals over all sites.  This reads the
 * integers N = sum_q b_q 2^q back out of the bit planes (Eqs. (15)-(19)), the
 * occupancies whose trajectories the paper plots (Sec. 5).  dev_dst is a
 * caller-owned device array of n_replicas * S int32.  Async. */
int bwg_ensemble_read_counts(bwg_ens *ens, int32_t *dev_dst, void *stream);

/* Histogram over replicas of the enantiomeric excess (N_L - N_D)/N_tot,
 * the chiral order parameter of the Frank model (Sec. 2; its spread over
 * copies is what the paper's trajectory figure shows, Sec. 5):
 * bin = min(n_bins-1, floor((N_L - N_D + N_tot) n_bins / (2 N_tot))),
 * dev_dst[n_bins] uint64 (overwritten).  Frank species only.  On a lattice
 * N_L, N_D are totals over sites and N_tot is the replica's molecule count
 * (a replica without molecules goes to bin n_bins/2).  Async. */
int bwg_ensemble_histogram(bwg_ens *ens, int32_t n_bins, uint64_t *dev_dst,
                           void *stream);

/* Trajectories of chosen replicas and first passages to homochirality (the
 * paper's trajectory figure and its use for rare events, Sec. 5 and Sec. 6):
 * for k = 0 .. n_points-1, advance to t_grid[k] (host array, non-decreasing,
 * from t_now on; EINVAL before any work otherwise), then
 *   - copy the counts of replicas dev_sel[0 .. n_sel) (device, uint32) into
 *     dev_out[(k * n_sel + j) * 3 + x] (device, int32, species order); an
 *     index at or past the replica count gives -1;
 *   - if dev_first is not NULL (device, uint32[n_replicas]): every replica
 *     whose entry is still 0xFFFFFFFF and whose |N_L - N_D| >= threshold gets
 *     dev_first[i] = k (the caller fills it with 0xFFFFFFFF first).
 * The same as n_points calls of bwg_ensemble_advance with a read after each.
 * Well-mixed ensembles of any engine, Frank species (EUNSUPPORTED for
 * lattices).  Async. */
int bwg_ensemble_record(bwg_ens *ens, const double *t_grid, uint32_t n_points,
                        const uint32_t *dev_sel, uint32_t n_sel, int32_t *dev_out,
                        int32_t threshold, uint32_t *dev_first, void *stream);

/* Events run per replica, dev_events[i], and real (state-changing) events
 * so far, dev_real[]: per replica for the plain engine, per 32-replica word
 * (ceil(M/32) entries) for the bit-sliced engine and lattices.  uint64;
 * either pointer may be NULL.  Async. */
int bwg_ensemble_read_events(bwg_ens *ens, uint64_t *dev_events,
                             uint64_t *dev_real, void *stream);

/* Lattice ensembles: site counts of replicas first .. first+count-1,
 * dev_dst[(k*sites + s)*3 + x] int32 (species L, D, A).  EINVAL for a
 * well-mixed ensemble or a range beyond the replicas.  Async. */
int bwg_ensemble_read_sites(bwg_ens *ens, uint64_t first, uint64_t count, int32_t *dev_dst,
                            void *stream);

/* Lattice ensembles: hops into full sites so far, per 32-replica word,
 * dev_dst[ceil(M/32)] uint64.  Async. */
int bwg_ensemble_read_blocked(bwg_ens *ens, uint64_t *dev_dst, void *stream);

/* With BWG_OPT_TIME_KERNELS: waits for the event-kernel launches enqueued
 * since the last call (wm_event_kernel, plain_event_kernel or
 * lat_event_kernel; not the budget, schedule or readout kernels) and
 * returns their summed duration in ms, measured with HIP events on the
 * launch stream, and their number; then starts a new count.  EINVAL if the
 * ensemble was created without the flag. */
int bwg_ensemble_kernel_time(bwg_ens *ens, double *ms, uint64_t *launches);

/* Switch an ensemble between BWG_ENGINE_BITWISE and BWG_ENGINE_LANES (same
 * state layout and random draws, so results do not change); EINVAL for other
 * engines, lattices or a plain ensemble.  Takes effect at the next launch. */
int bwg_ensemble_set_engine(bwg_ens *ens, int32_t engine);

/* Builds now the kernel that the ensemble's next bit-sliced launch would
 * compile at run time (a Frank-family network on a run-time weight variant,
 * see BWG_OPT_NO_JIT), so that the compile does not fall into a later launch
 * (a timed region, a serving loop); shared by every ensemble of the network.
 * A no-op for every other ensemble.  EDEVICE if the compile fails, EINVAL
 * for a null ensemble.  Host only. */
int bwg_ensemble_prepare(bwg_ens *ens);

/* Checkpoint and resume between advances.  Every draw is keyed by replica,
 * absolute event index and advance index (counter-based, Sec. 3 and Sec. 4
 * draws of the chain), so the counts, the event counters, t_now and the
 * advance index fix the rest of a run: an ensemble restored from a
 * checkpoint and advanced further gives, bit for bit, what the saved one
 * would have given, if both have the same seed and net_id (with others it
 * continues from the saved state on other draws).
 *
 * bwg_ensemble_checkpoint_bytes: host bytes a checkpoint of ens takes.
 * bwg_ensemble_save: copy the state into host_dst (caller-owned, dst_bytes
 *   at least that size; ERANGE otherwise); EINVAL before init or while
 *   events of the last advance or step are pending.  Synchronous: returns
 *   after the copies on stream have finished.
 * bwg_ensemble_restore: load a checkpoint into ens, which must be created
 *   for the same network (the same integer form), replica count and state
 *   kind (bit planes -- the BITWISE and LANES engines share them --, PLAIN
 *   counts, or lattice) and shared-threshold option; other options may
 *   differ.  EINVAL for anything else, for replicas with pending events or a
 *   shared-threshold checkpoint whose replicas are not at one event; ERANGE
 *   for an event index of 2^47 or more.  Synchronous.
 *
 * Layout (host byte order; the first 256 bytes are 32 uint64 header words):
 *   [0] magic 0x31544b5043475742, [1] header bytes (256), [2] total bytes,
 *   [3] network fingerprint (FNV-1a of the integer form), [4] n_replicas,
 *   [5] seed, [6] net_id, [7] state kind (0 bit planes, 1 plain, 2 lattice),
 *   [8] shared-threshold range Z (0: none), [9] t_now (binary64 bits),
 *   [10] advance index, [11] region count r (<= 6), then for k < r the words
 *   [12+3k] region id, [13+3k] byte offset (a multiple of 256), [14+3k] bytes.
 * Region ids: 1 bit planes (the device layout: [species][plane][word]
 * uint32, lattices [group][site][species][plane] words), 2 plain counts
 * (int32 [replica][3]), 3 events run per replica (uint64; entries past
 * n_replicas up to the padded word count are ignored), 4 event targets
 * (uint64, equal to region 3 between advances), 5 real events (uint64, per
 * 32-replica word, per replica for PLAIN), 6 blocked hops (uint64 per word,
 * lattices). */
int bwg_ensemble_checkpoint_bytes(const bwg_ens *ens, uint64_t *bytes);
int bwg_ensemble_save(bwg_ens *ens, void *host_dst, uint64_t dst_bytes, void *stream);
int bwg_ensemble_restore(bwg_ens *ens, const void *host_src, uint64_t src_bytes, void *stream);

/* In batches, run the last n_words words of a bit-sliced ensemble (rounded so
 * that the bit-sliced part is whole 64-word items) as lanes items of the same
 * persistent launch: the two kinds of item fill the SIMDs that one wave per
 * 64 words would leave idle.  Results do not change.  The ensemble's own
 * launches are not affected.  EINVAL for lattices and the plain engine. */
int bwg_ensemble_set_lanes_words(bwg_ens *ens, uint64_t n_words);

/* Synchronises the stream and reports totals. */
int bwg_ensemble_stats(bwg_ens *ens, void *stream, bwg_stats *out);

/* ---- allocation-free run ------------------------------------------------ */

/* Bytes of the library's static device array that holds the state of a
 * bwg_ensemble_step_static run (one array per GPU, held until the process
 * ends). */
#define BWG_STATIC_STATE_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid allocation): the same as
 * creating a bit-sliced ensemble of n_replicas of a well-mixed network
 * (seed, net_id), bwg_ensemble_init(BWG_INIT_FIXED, counts), bwg_ensemble_step
 * (n_events) and bwg_ensemble_read_counts(dev_counts), with the ensemble's
 * device state in the library's static array instead of a caller buffer and
 * the precompiled kernels only (BWG_OPT_NO_JIT): the results are those of
 * that sequence.  counts[S] is a host array summing to n_tot; dev_counts is a
 * caller-owned device array of n_replicas * S int32 (species order of the
 * network).  No device or pinned memory is allocated and nothing is
 * compiled.  ERANGE if the state of n_replicas exceeds BWG_STATIC_STATE_BYTES
 * (e.g. about 3 * 10^6 replicas at 11 count planes); EUNSUPPORTED for
 * lattices.  Every call on one GPU uses that GPU's one array, so calls that
 * overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller; a call leaves its state in the array, and the
 * next call rewrites every word it reads before reading it.  Async. */
int bwg_ensemble_step_static(const bwg_net *net, uint64_t n_replicas, uint64_t seed,
                             uint32_t net_id, const int32_t *counts, uint64_t n_events,
                             int32_t *dev_counts, void *stream);

void bwg_ensemble_destroy(bwg_ens *ens);

/* ---- batches: many ensembles in one persistent launch ------------------- */

typedef struct bwg_batch bwg_batch;

typedef struct {
    int32_t waves;          /* persistent grid in wavefronts, 0 = default (2048)  */
    int32_t order;          /* 0: longest pending work first, 1: member order     */
    int32_t max_ensembles;  /* capacity for later member changes (0: initial n)   */
    int32_t reserved0;
    uint64_t max_items;     /* capacity in 64-word work items (0: initial)        */
    uint64_t reserved[3];
} bwg_batch_opts;

/* Device bytes the batch bookkeeping needs (queue, descriptors) for exactly
 * these members, or for a capacity of members and 64-word work items. */
int bwg_batch_state_bytes(bwg_ens *const *ens, int32_t n, uint64_t *bytes);
int bwg_batch_capacity_bytes(int32_t max_ensembles, uint64_t max_items, uint64_t *bytes);

/* Group n bit-sliced ensembles (distinct, possibly of different networks,
 * sizes and plane widths) so that one launch advances all of them.  The
 * ensembles stay usable on their own.  Synchronises the stream once.
 * EUNSUPPORTED if an ensemble's planes fit no bucket of the persistent
 * kernel. */
int bwg_batch_create(bwg_ens *const *ens, int32_t n, void *dev_buf, uint64_t buf_bytes,
                     const bwg_batch_opts *opts, void *stream, bwg_batch **out);

/* Replace the members (within the capacity; ERANGE beyond it).  Members'
 * scheduled but unrun events stay pending in the ensembles.  Async. */
int bwg_batch_set_members(bwg_batch *b, bwg_ens *const *ens, int32_t n, void *stream);

/* One persistent launch over every member's pending events, at most
 * max_events per word (0: all).  Async. */
int bwg_batch_run(bwg_batch *b, uint64_t max_events, void *stream);

/* Advance ensemble k to t_end[k] (host array of n).  Every replica's result
 * is identical to a bwg_ensemble_advance of its ensemble alone: the draws are
 * keyed by (seed, net_id, replica, event), not by launch or order.  Async. */
int bwg_batch_advance(bwg_batch *b, const double *t_end, void *stream);

/* Capture one advance of every ensemble by dt into a HIP graph and replay it
 * n_steps times (the advance index lives on the device, so each replay draws
 * new budgets).  EINVAL unless t + dt - t == dt exactly in binary64 for every
 * step of every ensemble (each replay then has the same Poisson mean).
 * Synchronises the stream at the end. */
int bwg_batch_graph_advance(bwg_batch *b, double dt, int32_t n_steps, void *stream);

void bwg_batch_destroy(bwg_batch *b);

const char *bwg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BWG_H */
