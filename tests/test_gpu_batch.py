"""Batched persistent execution and graph replays, through the C ABI.

A replica's result may not depend on which launch, queue order, grid size or
graph replay ran it: every test compares bit for bit with each ensemble
advanced alone, and the small cases with the CPU oracle.
"""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from workloads import batch_networks, frank_network

pytestmark = pytest.mark.gpu

MIX = [  # (network, replicas, t_end) of uneven sizes and plane widths
    (frank_network(16, k0=0.05), 33, 12.0),
    (frank_network(100, k0=0.01), 1000, 3.0),
    (frank_network(300, k0=0.003), 2048, 1.5),
    (frank_network(1000, k0=0.02), 97, 0.75),
    (frank_network(40, k0=0.1), 5000, 6.0),
    (frank_network(2000, k0=0.001), 64, 0.25),
    (frank_network(3000, k0=0.07), 130, 0.2),
]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _say(*a):
    print(*a, flush=True)


def _ensembles(mix, seed=3):
    out = []
    for k, (net, M, _) in enumerate(mix):
        e = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=100 + k)
        e.init_fixed((0, 0, net["n_tot"]))
        out.append(e)
    return out


def _state(torch, ens):
    c = [e.read_counts() for e in ens]
    ev = [e.read_events()[0] for e in ens]
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in c], [x.cpu().numpy() for x in ev]


def _assert_same(a, b):
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y)
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y)


def test_batch_equals_each_ensemble_alone(torch):
    _say("case batch-vs-alone", len(MIX))
    batched = _ensembles(MIX)
    alone = _ensembles(MIX)
    b = bwg.Batch(batched)
    t1 = [t for _, _, t in MIX]
    t2 = [2.5 * t for _, _, t in MIX]
    b.advance(t1)
    b.advance(t2)
    for e, x, y in zip(alone, t1, t2):
        e.advance(x)
        e.advance(y)
    _assert_same(_state(torch, batched), _state(torch, alone))


def test_batch_matches_oracle(torch):
    _say("case batch-vs-oracle")
    mix = MIX[:2] + MIX[4:5]
    batched = _ensembles(mix, seed=9)
    b = bwg.Batch(batched)
    b.advance([t for _, _, t in mix])
    counts, ev = _state(torch, batched)
    for k, (net, M, t) in enumerate(mix):
        o = ssa.OracleEnsemble(net, M, seed=9, net_id=100 + k)
        o.init(("fixed", (0, 0, net["n_tot"])))
        o.advance(t)
        np.testing.assert_array_equal(counts[k], o.counts)
        np.testing.assert_array_equal(ev[k].astype(np.uint64), o.E)


@pytest.mark.parametrize("waves,order", [(64, 0), (200, 1), (4096, 0)])
def test_queue_order_and_grid_do_not_change_results(torch, waves, order):
    _say("case grid", waves, order)
    ref = _ensembles(MIX)
    bwg.Batch(ref).advance([t for _, _, t in MIX])
    other = _ensembles(MIX)
    bwg.Batch(other, waves=waves, order=order).advance([t for _, _, t in MIX])
    _assert_same(_state(torch, ref), _state(torch, other))


def test_graph_replays_equal_sequential_advances(torch):
    _say("case graph")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = _ensembles(MIX, seed=5)
        b = bwg.Batch(g)
        b.graph_advance(0.125, 6)
        seq = _ensembles(MIX, seed=5)
        for step in range(1, 7):
            for e in seq:
                e.advance(0.125 * step)
        st_g, st_s = _state(torch, g), _state(torch, seq)
    torch.cuda.synchronize()
    _assert_same(st_g, st_s)
    assert all(e.stats()["advance_index"] == 6 for e in g)


def test_graph_rejects_inexact_steps(torch):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = bwg.Batch(_ensembles(MIX[:2]))
        with pytest.raises(bwg.BwgError):
            b.graph_advance(0.1, 50)     # t + 0.1 - t != 0.1 somewhere


def test_uneven_batch_workload_sample(torch):
    # the first 24 networks of the uneven batch, replicas capped at 2^12 and
    # horizons scaled down so the standalone comparison stays short
    cfg = batch_networks()[:24]
    mix = [(c["net"], min(c["replicas"], 4096), c["t_end"] / 200.0) for c in cfg]
    _say("case uneven sample", len(mix))
    batched = _ensembles(mix, seed=0)
    alone = _ensembles(mix, seed=0)
    bwg.Batch(batched).advance([t for _, _, t in mix])
    for e, (_, _, t) in zip(alone, mix):
        e.advance(t)
    _assert_same(_state(torch, batched), _state(torch, alone))


def test_full_uneven_batch_first_words_match_oracle(torch):
    """The whole uneven batch (256 networks, full replica counts and
    horizons) in one persistent launch: the first two words (64 replicas)
    of every network against the oracle, counts and events per replica."""
    cfg = batch_networks()
    _say("case full uneven batch", len(cfg))
    ens = []
    for c in cfg:
        e = bwg.Ensemble(bwg.Network(c["net"]), c["replicas"], seed=c["seed"],
                         net_id=c["net_id"])
        e.init(c["init"])
        ens.append(e)
    bwg.Batch(ens).advance([c["t_end"] for c in cfg])
    first = [(e.read_counts()[:64].cpu().numpy(), e.read_events()[0][:64].cpu().numpy())
             for e in ens]
    torch.cuda.synchronize()
    bad = []
    for k, (c, (gc, ge)) in enumerate(zip(cfg, first)):
        n = min(64, c["replicas"])
        o = ssa.OracleEnsemble(c["net"], c["replicas"], seed=c["seed"], net_id=c["net_id"],
                               first=0, count=n)
        o.init(c["init"])
        o.advance(c["t_end"])
        if not (np.array_equal(gc[:n], o.counts) and np.array_equal(ge[:n].astype(np.uint64), o.E)):
            bad.append(k)
    assert not bad, "networks whose first words differ from the oracle: %s" % bad[:16]


def test_batch_with_lanes_members_equals_alone(torch):
    """Members on the lanes engine (2-word items, one replica per thread)
    beside bit-sliced members give the same results as each alone."""
    mix = MIX[:6]
    alone = _ensembles(mix, seed=8)
    for e, (_, _, t) in zip(alone, mix):
        e.advance(t)
    ref = _state(torch, alone)
    ens = _ensembles(mix, seed=8)
    for k in (0, 3, 5):
        ens[k].set_engine("lanes")
    b = bwg.Batch(ens, waves=512)
    b.advance([t for _, _, t in mix])
    _assert_same(_state(torch, ens), ref)
    # and capped passes
    ens = _ensembles(mix, seed=8)
    for k in (1, 3):
        ens[k].set_engine("lanes")
    b = bwg.Batch(ens, waves=256)
    for e, (_, _, t) in zip(ens, mix):
        e.schedule(t)
    while any(e.pending() for e in ens):
        b.run(400)
    _assert_same(_state(torch, ens), ref)


def test_split_members_equal_alone(torch):
    """A bit-sliced member whose trailing words run as lanes items of the same
    persistent launch gives the same results."""
    net = frank_network(300, k0=0.003)
    M = 64 * 32 * 3 + 45          # 3 whole 64-word items and a ragged tail
    alone = bwg.Ensemble(bwg.Network(net), M, seed=6, net_id=44)
    alone.init_fixed((0, 0, 300)).advance(2.0)
    ref = _state(torch, [alone])
    for lw in (1, 64, 100, 10 ** 6):
        e = bwg.Ensemble(bwg.Network(net), M, seed=6, net_id=44)
        e.init_fixed((0, 0, 300))
        e.set_lanes_words(lw)
        bwg.Batch([e], waves=300).advance([2.0])
        _assert_same(_state(torch, [e]), ref)
