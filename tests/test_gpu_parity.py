"""GPU path against the CPU oracle, through the C ABI.

Every comparison is bit-exact: counts of every replica, events run per
replica and real (state-changing) events per 32-lane group.  Both sides use
the same seeded inputs and the same draw contract; they share no code.
"""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from oracle.poisson import poisson_table
from oracle.quantize import quantize
from workloads import config, frank_network, paper_network

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _say(*a):
    print(*a, flush=True)


def gpu_run(torch, net, M, init, schedule, seed=0, net_id=0, engine="bitwise", epl=0,
            shared=False, block=0, jit=True):
    n = bwg.Network(net)
    ens = bwg.Ensemble(n, M, seed=seed, net_id=net_id, engine=engine, events_per_launch=epl,
                       shared_threshold=shared, block=block, jit=jit)
    ens.init(init)
    for op, v in schedule:
        if op == "advance":
            ens.advance(v)
        else:
            ens.step(v)
    counts = ens.read_counts()
    ev, real = ens.read_events()
    torch.cuda.synchronize()
    return (counts.cpu().numpy(), ev.cpu().numpy().astype(np.uint64),
            real.cpu().numpy().astype(np.uint64), ens)


def oracle_run(net, M, init, schedule, seed=0, net_id=0, draw=ssa.DRAW_EVENT, first=0,
               count=None):
    E = ssa.OracleEnsemble(net, M, seed=seed, net_id=net_id, draw=draw, first=first,
                           count=count)
    E.init(init)
    for op, v in schedule:
        if op == "advance":
            E.advance(v)
        else:
            E.step(v)
    return E


def group_sums(x, M):
    g = (M + 31) // 32
    out = np.zeros(g, dtype=np.uint64)
    np.add.at(out, np.arange(M) // 32, x.astype(np.uint64))
    return out


def check_parity(torch, net, M, init, schedule, seed=0, net_id=0, engine="bitwise", epl=0,
                 shared=False, block=0, jit=True):
    _say("case", engine, net["n_tot"], M, init, schedule, seed, net_id, epl, shared, block, jit)
    counts, ev, real, ens = gpu_run(torch, net, M, init, schedule, seed, net_id, engine, epl,
                                    shared, block, jit)
    draw = (ssa.DRAW_PLAIN if engine == "plain" else
            ssa.DRAW_SHARED if shared else ssa.DRAW_EVENT)
    o = oracle_run(net, M, init, schedule, seed, net_id, draw)
    np.testing.assert_array_equal(counts, o.counts)
    np.testing.assert_array_equal(ev, o.E)
    if engine != "plain":
        np.testing.assert_array_equal(real, group_sums(o.real, M))
    else:
        np.testing.assert_array_equal(real, o.real)
    assert (counts.sum(1) == net["n_tot"]).all()
    return counts, ens


# ---- bit-sliced engine --------------------------------------------------------

def test_small_well_mixed_workload_exact(torch):
    c = config("c0")
    counts, ens = check_parity(torch, c["net"], c["replicas"], c["init"],
                               [("advance", c["t_end"])])
    h = ens.histogram(256).cpu().numpy()
    np.testing.assert_array_equal(h, ssa.ee_histogram(counts, 32, 256).astype(np.int64))
    s = ens.stats()
    assert s["advance_index"] == 1 and s["t_now"] == 50.0


def test_ragged_replicas_and_several_advances(torch):
    check_parity(torch, frank_network(32), 1000, ("fixed", (0, 0, 32)),
                 [("advance", 10.0), ("advance", 25.0), ("advance", 25.0), ("advance", 50.0)],
                 seed=7, net_id=3)


@pytest.mark.parametrize("M", [1, 31, 33, 65])
def test_partial_words(torch, M):
    check_parity(torch, frank_network(32), M, ("fixed", (4, 3, 25)),
                 [("advance", 20.0), ("step", 300)], seed=11, net_id=1)


def test_events_per_launch_chunking(torch):
    net = frank_network(32)
    sched = [("advance", 15.0), ("advance", 40.0)]
    check_parity(torch, net, 2048, ("fixed", (0, 0, 32)), sched, seed=5, epl=97)
    a = gpu_run(torch, net, 2048, ("fixed", (0, 0, 32)), sched, seed=5, epl=0)
    b = gpu_run(torch, net, 2048, ("fixed", (0, 0, 32)), sched, seed=5, epl=1)
    np.testing.assert_array_equal(a[0], b[0])


def test_per_event_trajectories(torch):
    # state after every single event equals the oracle's trajectory
    net = frank_network(32, k0=0.05)
    M, K = 96, 150
    n = bwg.Network(net)
    ens = bwg.Ensemble(n, M, seed=2, net_id=9)
    ens.init_fixed((10, 12, 10))
    states = []
    for _ in range(K):
        ens.step(1)
        states.append(ens.read_counts().cpu().numpy())
    torch.cuda.synchronize()
    q = quantize(net)
    counts0 = np.tile(np.array([10, 12, 10], np.int32), (M, 1))
    _, _, traj = ssa.run_events(net, q, 2, 9, 0, counts0, np.zeros(M, np.uint64),
                                np.full(M, K, np.uint64), traj_len=K)
    for t in range(K):
        np.testing.assert_array_equal(states[t], traj[:, t, :])


def test_paper_network_multinomial_start(torch):
    c = config("c0p")
    check_parity(torch, c["net"], 4096, ("multinomial",), [("step", 3000)], seed=1)


# Frank networks whose weights match no precompiled variant: by default the
# kernels compiled for the network (hipRTC), with jit=False the precompiled
# run-time weight kernels; both against the oracle.
@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("n_tot,k0", [(12, 0.01), (40, 0.05), (100, 0.01), (300, 0.002),
                                      (1000, 0.02), (16, 0.1), (3, 0.1), (7, 0.1)])
def test_run_time_shift_kernels(torch, n_tot, k0, jit):
    net = frank_network(n_tot, k0=k0)
    check_parity(torch, net, 700, ("fixed", (0, 0, n_tot)), [("advance", 3.0)], seed=4,
                 net_id=n_tot, jit=jit)


# Frank networks whose L + D rate differs from the A + L / A + D rate: the two
# product shifts differ (k2 = k1 / 4: the L + D weight is 2^(f-2) P_LD;
# k2 = 2 k1: the A + L, A + D weights are 2^(f-1) P), so the L + D
# subtraction must use its own shift in the compiled kernels (per-replica,
# producer/consumer and shared-threshold forms) and in the precompiled
# run-time kernels alike.
@pytest.mark.parametrize("shared,block", [(False, 0), (False, 128), (True, 0)])
@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("n_tot,k0,r2", [(64, 0.01, 0.25), (64, 0.01, 2.0), (300, 0.002, 0.25),
                                         (1000, 0.02, 2.0), (40, 0.05, 1.0)])
def test_unequal_product_shifts(torch, n_tot, k0, r2, jit, shared, block):
    net = frank_network(n_tot, k0=k0, k2=r2 / n_tot)
    q = bwg.Network(net).quantized()
    c = q["c"]
    assert (c[4] == 2 * c[2]) if r2 == 2.0 else (c[2] == 4 * c[4]) if r2 == 0.25 else c[2] == c[4]
    check_parity(torch, net, 700, ("multinomial",), [("advance", 2.0), ("step", 50)], seed=14,
                 net_id=n_tot + 1, jit=jit, shared=shared, block=block)


# The compiled kernel in its one-wave-per-word form (more than 32768 words,
# 256-thread blocks from 65536 on) against the precompiled run-time weight
# kernel, which the oracle pins above: every count and event counter equal.
# With shared thresholds the compiled kernel is the shared-threshold
# instantiation (one wave per word at any size).
@pytest.mark.parametrize("M,shared,r2", [((1 << 20) + (1 << 16) + 5, False, 1.0),
                                         ((1 << 21) + 33, False, 1.0),
                                         ((1 << 20) + (1 << 16) + 5, False, 0.25),
                                         (4096 + 7, True, 1.0), ((1 << 20) + 33, True, 1.0),
                                         ((1 << 20) + 33, True, 2.0)])
def test_compiled_frank_kernel_equals_precompiled(torch, M, shared, r2):
    net = frank_network(1024, k0=0.02, k2=r2 / 1024)
    sched = [("step", 300), ("step", 77)] if shared else [("advance", 0.4), ("step", 77)]
    a = gpu_run(torch, net, M, ("multinomial",), sched, seed=8, net_id=5, shared=shared, jit=True)
    b = gpu_run(torch, net, M, ("multinomial",), sched, seed=8, net_id=5, shared=shared,
                jit=False)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_pure_conversion_without_bimolecular_reactions(torch):
    net = frank_network(20, k0=0.05, k1=0.0, k2=0.0)
    check_parity(torch, net, 512, ("fixed", (0, 0, 20)), [("advance", 5.0)], seed=12)


def test_paper_network_without_ghosts(torch):
    net = paper_network(24, ghosts=False)
    check_parity(torch, net, 256, ("multinomial",), [("step", 1000)], seed=13)


def test_zero_length_advance_is_a_no_op(torch):
    net = frank_network(32)
    a = gpu_run(torch, net, 128, ("fixed", (0, 0, 32)), [("advance", 5.0)], seed=3)
    b = gpu_run(torch, net, 128, ("fixed", (0, 0, 32)), [("advance", 5.0), ("advance", 5.0)],
                seed=3)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_deterministic_reruns(torch):
    net = frank_network(64)
    a = gpu_run(torch, net, 4096, ("fixed", (0, 0, 64)), [("advance", 30.0)], seed=21)
    b = gpu_run(torch, net, 4096, ("fixed", (0, 0, 64)), [("advance", 30.0)], seed=21)
    np.testing.assert_array_equal(a[0], b[0])


def test_error_paths(torch):
    n = bwg.Network(frank_network(32))
    ens = bwg.Ensemble(n, 64)
    with pytest.raises(bwg.BwgError):
        ens.advance(1.0)          # not initialised
    ens.init_fixed((0, 0, 32))
    ens.advance(2.0)
    with pytest.raises(bwg.BwgError):
        ens.advance(1.0)          # backwards in time
    with pytest.raises(bwg.BwgError):
        ens.init_fixed((0, 0, 31))  # does not sum to N_tot
    with pytest.raises(bwg.BwgError):
        ens.histogram(0)


# ---- the two forms of the bit-sliced word kernel ----------------------------
# With the default block and at most 32768 words a launch runs the producer/
# consumer form (per 128 words two waves draw threshold planes into LDS and
# two run the events); an explicit block size selects the one-wave-per-word
# form.  The cases cover partial workgroups, a workgroup whose second group
# of 64 words is empty, and words with different event windows.

@pytest.mark.parametrize("block", [0, 64, 128, 256])
@pytest.mark.parametrize("net,M,init,sched,epl", [
    (frank_network(32), 64 * 32 * 3 + 17, ("fixed", (0, 0, 32)), [("advance", 30.0)], 0),
    (frank_network(1024), 4096 + 5, ("fixed", (0, 0, 1024)), [("advance", 0.4), ("step", 99)], 0),
    (paper_network(100), 31, ("multinomial",), [("step", 2500)], 333),
    (frank_network(200, k0=0.03), 2048, ("multinomial",), [("advance", 2.0), ("advance", 2.5)], 1000),
])
def test_word_kernel_forms_match_oracle(torch, block, net, M, init, sched, epl):
    check_parity(torch, net, M, init, sched, seed=12, net_id=4, epl=epl, block=block)


# The active lanes of a word change only where one of its replicas starts or
# ends its budget; the kernels rebuild the set at exactly those events.  After
# each short advance the replicas of a word stand at different event counts,
# so every later launch has lanes starting and ending at different events of
# the same word (both forms of the word kernel, ragged last word, two
# workgroups of the producer/consumer form).
@pytest.mark.parametrize("block", [0, 128])
def test_staggered_starts_and_ends(torch, block):
    net = frank_network(200, k0=0.03)
    q = bwg.Network(net).quantized()
    dt = 60.0 / q["Lambda"]                   # about 60 events per replica
    sched = [("advance", dt * (k + 1)) for k in range(20)]
    check_parity(torch, net, 64 * 32 * 2 + 45, ("multinomial",), sched, seed=21, net_id=6,
                 block=block)


# ---- comparator engine -----------------------------------------------------------

def test_plain_engine_exact(torch):
    c = config("c0")
    check_parity(torch, c["net"], c["replicas"], c["init"], [("advance", c["t_end"])],
                 engine="plain")


def test_plain_engine_ragged_and_multinomial(torch):
    check_parity(torch, paper_network(32), 777, ("multinomial",), [("step", 2000)], seed=8,
                 engine="plain")
    check_parity(torch, frank_network(100), 333, ("fixed", (0, 0, 100)),
                 [("advance", 2.0), ("advance", 7.0)], seed=9, engine="plain", epl=50)


# ---- full-size workload -----------------------------------------------------------

def test_full_size_well_mixed_workload_sampled(torch):
    # N_tot = 1024, 2^20 replicas, t_end = 100 in one launch: exact parity on
    # sampled replicas, exact event counts for every replica, conservation
    # and histogram mass for all.
    c = config("c1")
    net, M = c["net"], c["replicas"]
    _say("case full-size", M)
    counts, ev, real, ens = gpu_run(torch, net, M, c["init"], [("advance", c["t_end"])])
    hist = ens.histogram(256).cpu().numpy()
    assert (counts.sum(1) == 1024).all() and (counts >= 0).all()
    assert hist.sum() == M
    np.testing.assert_array_equal(hist, ssa.ee_histogram(counts, 1024, 256).astype(np.int64))
    q = quantize(net)
    table = poisson_table(q["Lambda"] * c["t_end"])
    K = ssa.budgets(0, 0, 0, 0, M, table)
    np.testing.assert_array_equal(ev, K)
    # the first 2^14 replicas (512 words: four producer/consumer workgroups)
    # and blocks spread over the rest, counts and events per replica
    for first, count in ((0, 1 << 14), (1 << 19, 64), (M - 64, 64), (777 * 32 + 5, 16)):
        E = ssa.OracleEnsemble(net, M, first=first, count=count)
        E.init(c["init"])
        E.advance(c["t_end"])
        np.testing.assert_array_equal(counts[first:first + count], E.counts)
        np.testing.assert_array_equal(ev[first:first + count], E.E)


# ---- lanes engine: one replica per thread on the bit-plane state ------------

@pytest.mark.parametrize("n_tot,M,sched", [
    (32, 1024, [("advance", 50.0)]),
    (100, 1000, [("advance", 2.0), ("advance", 5.5)]),
    (1024, 333, [("step", 3000)]),
    (12, 65, [("advance", 40.0), ("step", 77)]),
])
def test_lanes_engine_matches_oracle(torch, n_tot, M, sched):
    check_parity(torch, frank_network(n_tot), M, ("fixed", (0, 0, n_tot)), sched, seed=4,
                 net_id=3, engine="lanes")


def test_lanes_engine_paper_network_and_chunking(torch):
    check_parity(torch, paper_network(32), 200, ("multinomial",), [("step", 4000)], seed=2,
                 engine="lanes")
    check_parity(torch, frank_network(64), 97, ("fixed", (0, 0, 64)), [("advance", 8.0)],
                 engine="lanes", epl=700)


def test_switching_engines_mid_run_changes_nothing(torch):
    net = frank_network(200, k0=0.03)
    M = 2000
    a = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=1)
    b = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=1, engine="lanes")
    for e in (a, b):
        e.init_fixed((0, 0, 200))
    a.advance(1.0)
    b.advance(1.0)
    b.set_engine("bitwise")
    a.set_engine("lanes")
    a.schedule(3.0)
    b.schedule(3.0)
    while a.pending() or b.pending():
        a.run(500)
        b.run(300)
    for x, y in ((a.read_counts(), b.read_counts()), (a.read_events()[0], b.read_events()[0]),
                 (a.read_events()[1], b.read_events()[1])):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(bwg.Network(net), 10, engine="plain").set_engine("lanes")


# ---- shared threshold: one n on [0, Z) for every replica (Sec. 4) ----------

@pytest.mark.parametrize("net,M,init,sched,engine,epl", [
    (paper_network(32), 1000, ("multinomial",), [("step", 3000)], "bitwise", 0),
    (paper_network(100), 333, ("fixed", (30, 30, 40)), [("step", 5000)], "lanes", 0),
    (paper_network(32), 200, ("multinomial",), [("step", 1500), ("step", 7)], "lanes", 700),
    (paper_network(1024), 97, ("multinomial",), [("step", 2000)], "bitwise", 500),
    (frank_network(64), 700, ("fixed", (0, 0, 64)), [("step", 2000), ("step", 77)], "bitwise", 0),
    (frank_network(12), 65, ("fixed", (0, 0, 12)), [("step", 900)], "lanes", 0),
])
def test_shared_threshold_matches_oracle(torch, net, M, init, sched, engine, epl):
    """Z = N(N-1)/2 for the paper's network with ghosts, Z = W without them."""
    check_parity(torch, net, M, init, sched, seed=6, net_id=9, engine=engine, epl=epl,
                 shared=True)


def test_shared_threshold_launches_and_capped_runs(torch):
    """Steps longer than the threshold table (2 x table_capacity events) run
    in several fill + event launches; events_per_launch caps them further."""
    net = paper_network(48)
    for kw in (dict(table_capacity=1000), dict(table_capacity=4096, events_per_launch=777)):
        n = bwg.Network(net)
        e = bwg.Ensemble(n, 300, seed=8, net_id=2, shared_threshold=True, **kw)
        e.init(("multinomial",))
        e.step(5001)
        e.step(3)
        o = oracle_run(net, 300, ("multinomial",), [("step", 5001), ("step", 3)], seed=8,
                       net_id=2, draw=ssa.DRAW_SHARED)
        np.testing.assert_array_equal(e.read_counts().cpu().numpy(), o.counts)
        np.testing.assert_array_equal(e.read_events()[0].cpu().numpy(), o.E)


def test_shared_threshold_copies_from_one_state_stay_equal(torch):
    net = paper_network(64)
    counts, _, _, _ = gpu_run(torch, net, 3000, ("fixed", (20, 20, 24)), [("step", 4000)],
                              seed=1, shared=True)
    assert (counts == counts[0]).all()


def test_shared_threshold_full_size_sampled(torch):
    """The gain workload's launch: the paper's network at N = 1024 with its
    ghosts, 2^22 replicas from a multinomial start, 10^5 steps (one table
    fill and one event launch); 3 blocks of 16 replicas against the oracle."""
    net = paper_network(1024)
    M, T = 1 << 22, 100000
    counts, ev, _, _ = gpu_run(torch, net, M, ("multinomial",), [("step", T)], seed=3,
                               net_id=1, shared=True)
    assert (ev == T).all()
    assert (counts.sum(1) == 1024).all()
    for first in (0, M // 2 + 5, M - 16):
        o = ssa.OracleEnsemble(net, M, seed=3, net_id=1, draw=ssa.DRAW_SHARED, first=first,
                               count=16)
        o.init(("multinomial",))
        o.step(T)
        np.testing.assert_array_equal(counts[first:first + 16], o.counts)


@pytest.mark.parametrize("net,M,sched,engine,epl,cap", [
    (paper_network(32), 1000, [("advance", 20.0)], "bitwise", 0, 0),
    (paper_network(100), 333, [("advance", 0.5), ("step", 77), ("advance", 1.25)], "lanes", 0, 0),
    (paper_network(64), 200, [("advance", 3.0), ("advance", 3.0), ("advance", 4.5)], "bitwise",
     700, 0),
    (paper_network(24), 97, [("advance", 40.0)], "bitwise", 0, 1000),
    (frank_network(64), 700, [("advance", 2.0), ("step", 10)], "bitwise", 0, 0),
])
def test_shared_time_matches_oracle(torch, net, M, sched, engine, epl, cap):
    """Advances of a shared-threshold ensemble: one budget for every replica
    at rate Z / s, run in launches of at most 2 x table_capacity events."""
    _say("shared time", net["n_tot"], M, sched, engine, epl, cap)
    n = bwg.Network(net)
    e = bwg.Ensemble(n, M, seed=5, net_id=8, engine=engine, events_per_launch=epl,
                     table_capacity=cap, shared_threshold=True)
    e.init(("multinomial",))
    o = ssa.OracleEnsemble(net, M, seed=5, net_id=8, draw=ssa.DRAW_SHARED)
    o.init(("multinomial",))
    for op, v in sched:
        getattr(e, op)(v)
        getattr(o, op)(v)
    ev, real = e.read_events()
    np.testing.assert_array_equal(e.read_counts().cpu().numpy(), o.counts)
    np.testing.assert_array_equal(ev.cpu().numpy(), o.E)
    np.testing.assert_array_equal(real.cpu().numpy().astype(np.uint64), group_sums(o.real, M))
    assert (o.E == o.E[0]).all() and o.E[0] > 0


def test_shared_time_split_schedule_and_run(torch):
    """schedule + capped runs give what one advance gives; a new schedule or
    step before the pending events have run is refused."""
    net = paper_network(40)
    a = bwg.Ensemble(bwg.Network(net), 500, seed=2, shared_threshold=True)
    b = bwg.Ensemble(bwg.Network(net), 500, seed=2, shared_threshold=True)
    for x in (a, b):
        x.init(("multinomial",))
    a.advance(5.0)
    b.schedule(5.0)
    b.run(333)
    with pytest.raises(bwg.BwgError):
        b.schedule(6.0)
    with pytest.raises(bwg.BwgError):
        b.step(5)
    while b.pending():
        b.run(333)
    np.testing.assert_array_equal(a.read_counts().cpu().numpy(), b.read_counts().cpu().numpy())
    np.testing.assert_array_equal(a.read_events()[0].cpu().numpy(),
                                  b.read_events()[0].cpu().numpy())


def test_shared_threshold_rejections(torch):
    net = bwg.Network(paper_network(32))
    e = bwg.Ensemble(net, 100, shared_threshold=True)
    e.init(("multinomial",))
    with pytest.raises(bwg.BwgError):
        bwg.Batch([e])
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(net, 100, engine="plain", shared_threshold=True)
    lat = bwg.Network(frank_network(12, lx=4, ly=4, hop=0.1, site_planes=4))
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(lat, 100, shared_threshold=True)
    e.step(10)                       # still usable after the refusals
    assert (e.read_events()[0].cpu().numpy() == 10).all()
