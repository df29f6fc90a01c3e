"""The general bit-sliced kernels (any 3-species network of order <= 2): the
per-network kernel compiled at run time and the precompiled one, against
the oracle, and against the Frank kernel on Frank networks."""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from workloads import frank_network, paper_network, random_network

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _group_sums(x, M):
    out = np.zeros((M + 31) // 32, dtype=np.uint64)
    np.add.at(out, np.arange(M) // 32, x.astype(np.uint64))
    return out


def _check(torch, net, M, init, sched, seed, net_id, generic=False, epl=0, jit=True):
    print("case", net["n_tot"], len(net["rates"]), M, init, sched, seed, generic, epl, jit,
          flush=True)
    e = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=net_id, generic=generic,
                     events_per_launch=epl, jit=jit)
    e.init(init)
    o = ssa.OracleEnsemble(net, M, seed=seed, net_id=net_id)
    o.init(init)
    for op, v in sched:
        getattr(e, op)(v)
        getattr(o, op)(v)
    ev, real = e.read_events()
    np.testing.assert_array_equal(e.read_counts().cpu().numpy(), o.counts)
    np.testing.assert_array_equal(ev.cpu().numpy().astype(np.uint64), o.E)
    np.testing.assert_array_equal(real.cpu().numpy().astype(np.uint64), _group_sums(o.real, M))
    return e


@pytest.mark.parametrize("seed,n_tot,R,M", [
    (0, 12, 3, 100), (1, 50, 7, 1000), (2, 200, 12, 333), (3, 12, 16, 65),
    (4, 30, 5, 2048 + 7), (5, 100, 9, 31), (6, 7, 4, 500), (7, 300, 6, 257), (8, 400, 5, 1024),
])
@pytest.mark.parametrize("jit", [True, False])
def test_random_networks_match_oracle(torch, seed, n_tot, R, M, jit):
    net = random_network(seed, n_tot, R)
    q = bwg.Network(net).quantized()
    mu_t = 400.0 / q["Lambda"]                # about 400 events per replica
    _check(torch, net, M, ("multinomial",), [("advance", mu_t), ("step", 123)], seed=seed,
           net_id=seed + 10, jit=jit)


# Many short advances: the replicas of a word start and end each launch at
# different events (the active lanes are rebuilt only where they change).
@pytest.mark.parametrize("jit", [True, False])
def test_staggered_starts_and_ends(torch, jit):
    net = random_network(9, 60, 6)
    q = bwg.Network(net).quantized()
    dt = 40.0 / q["Lambda"]                   # about 40 events per replica
    _check(torch, net, 64 * 32 * 2 + 45, ("multinomial",),
           [("advance", dt * (k + 1)) for k in range(15)], seed=9, net_id=19, jit=jit)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_random_integer_networks_match_oracle(torch, seed):
    net = random_network(seed, 40, 8, exact_integer=True)
    _check(torch, net, 700, ("multinomial",), [("step", 1500)], seed=seed, net_id=3, epl=400)


def test_one_compile_per_network(torch):
    """Ensembles of one network share its compiled kernel; equal results."""
    net = random_network(21, 60, 6)
    n = bwg.Network(net)
    a = bwg.Ensemble(n, 999, seed=2)
    b = bwg.Ensemble(n, 999, seed=2)
    for e in (a, b):
        e.init(("multinomial",)).step(700)
    np.testing.assert_array_equal(a.read_counts().cpu().numpy(), b.read_counts().cpu().numpy())


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("net", [frank_network(32), frank_network(1024), paper_network(64)])
def test_general_kernel_equals_frank_kernel(torch, net, jit):
    """Frank networks asked onto the general kernels give the Frank kernel's
    results (and the oracle's); the paper's network has trailing ghosts the
    run-time compiled kernel leaves out."""
    M = 1500
    sched = [("advance", 300.0 / bwg.Network(net).quantized()["Lambda"]), ("step", 50)]
    init = ("multinomial",)
    g = _check(torch, net, M, init, sched, seed=4, net_id=2, generic=True, jit=jit)
    f = bwg.Ensemble(bwg.Network(net), M, seed=4, net_id=2)
    f.init(init)
    for op, v in sched:
        getattr(f, op)(v)
    np.testing.assert_array_equal(g.read_counts().cpu().numpy(), f.read_counts().cpu().numpy())


def test_general_kernel_refusals(torch):
    net = random_network(0, 12, 3)
    e = bwg.Ensemble(bwg.Network(net), 64)
    e.init(("multinomial",))
    with pytest.raises(bwg.BwgError):
        e.set_engine("lanes")
    with pytest.raises(bwg.BwgError):
        bwg.Batch([e])
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(bwg.Network(net), 64, shared_threshold=True)


@pytest.mark.parametrize("jit", [True, False])
def test_large_ensemble_sampled(torch, jit):
    """Past 32768 words the compiled kernel runs one wave per word (below it
    the producer/consumer form): 2^20 + 77 replicas of a random network,
    three blocks of replicas against the oracle, including the ragged end."""
    net = random_network(31, 80, 6)
    M = (1 << 20) + 77
    e = bwg.Ensemble(bwg.Network(net), M, seed=6, net_id=4, jit=jit)
    e.init(("multinomial",)).step(300)
    counts = e.read_counts().cpu().numpy()
    for first, count in ((0, 64), (M // 2 - 5, 40), (M - 45, 45)):
        o = ssa.OracleEnsemble(net, M, seed=6, net_id=4, first=first, count=count)
        o.init(("multinomial",))
        o.step(300)
        np.testing.assert_array_equal(counts[first:first + count], o.counts)


# The compiled kernel's one-wave-per-word form with 256-thread blocks (from
# 65536 words) against the precompiled general kernel, which the oracle pins.
def test_compiled_kernel_large_blocks_equal_precompiled(torch):
    net = random_network(8, 400, 5)
    M = (1 << 21) + 5
    res = []
    for jit in (True, False):
        e = bwg.Ensemble(bwg.Network(net), M, seed=3, net_id=9, jit=jit)
        e.init(("multinomial",)).step(150)
        ev, real = e.read_events()
        res.append((e.read_counts().cpu().numpy(), ev.cpu().numpy(), real.cpu().numpy()))
    for x, y in zip(*res):
        np.testing.assert_array_equal(x, y)


def _table(reactions, rates, n_tot, integer=True):
    from workloads.frank import _net
    return _net(reactions, rates, n_tot, exact_integer=integer)


@pytest.mark.parametrize("jit", [True, False])
def test_edge_tables(torch, jit):
    """Zero weights between real reactions, a network where nothing changes
    the state, and a dimer conversion with a large weight."""
    zero_mid = _table([((0, 0, 1), (1, 0, 0)), ((1, 0, 0), (0, 1, 0)), ((0, 1, 0), (0, 0, 1)),
                       ((2, 0, 0), (0, 0, 2))], [3, 0, 2, 5], 20)
    still = _table([((1, 0, 0), (1, 0, 0)), ((0, 1, 1), (0, 1, 1))], [4, 1], 15)
    dimer = _table([((0, 0, 2), (1, 1, 0)), ((1, 1, 0), (0, 0, 2)), ((2, 0, 0), (1, 0, 1))],
                   [1000, 3, 7], 30)
    for net, init in ((zero_mid, ("fixed", (5, 5, 10))), (still, ("fixed", (5, 5, 5))),
                      (dimer, ("multinomial",))):
        e = _check(torch, net, 333, init, [("step", 800), ("step", 5)], seed=3, net_id=7, jit=jit)
    ev, real = e.read_events()
    assert int(real.sum()) > 0


def test_still_network_changes_nothing(torch):
    net = _table([((1, 0, 0), (1, 0, 0)), ((0, 1, 1), (0, 1, 1))], [4, 1], 15)
    e = bwg.Ensemble(bwg.Network(net), 100)
    e.init(("fixed", (5, 5, 5))).step(1000)
    assert (e.read_counts().cpu().numpy() == [5, 5, 5]).all()
    assert int(e.read_events()[1].sum()) == 0


def test_record_on_a_general_network(torch):
    net = random_network(41, 40, 6)
    M = 500
    grid = [0.2 * (k + 1) / bwg.Network(net).quantized()["Lambda"] * 100 for k in range(10)]
    e = bwg.Ensemble(bwg.Network(net), M, seed=2)
    e.init(("multinomial",))
    traj, first = e.record(grid, [0, 17, 499], threshold=10)
    o = ssa.OracleEnsemble(net, M, seed=2)
    o.init(("multinomial",))
    for k, t in enumerate(grid):
        o.advance(t)
        np.testing.assert_array_equal(traj[k].cpu().numpy(), o.counts[[0, 17, 499]])
