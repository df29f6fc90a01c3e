"""Ensembles at the largest replica counts the library takes.

n_replicas < 2^32: at 2^32 - 1 every per-replica launch (budgets, readouts,
the histogram, the lanes engine) needs two dispatches, since one dispatch
covers fewer than 2^32 work-items, and the last word holds 31 live
replicas.  The oracle runs sampled replicas one by one -- the first ones,
both sides of the dispatch boundary at 2^31 and the ragged tail -- and must
agree exactly; conservation, histogram mass and the histogram's bins are
checked over every replica.
"""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from oracle.poisson import poisson_table
from oracle.quantize import quantize
from workloads import frank_network

pytestmark = pytest.mark.gpu

M_MAX = (1 << 32) - 1
PIECE = 1 << 31
CHUNK = 1 << 28


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _say(*a):
    print(*a, flush=True)


def _need(torch, nbytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")


def _oracle(net, M, first, count, sched, draw):
    o = ssa.OracleEnsemble(net, M, first=first, count=count, draw=draw)
    o.init(("fixed", (0, 0, net["n_tot"])))
    for t in sched:
        o.advance(t)
    return o


def _check_all(torch, counts, n_tot, hist, n_bins):
    """Conservation over every replica and the histogram's bins from the
    counts, in chunks (a whole-array temporary would need tens of GB)."""
    M = counts.shape[0]
    ref = torch.zeros(n_bins, dtype=torch.int64, device=counts.device)
    for k in range(0, M, CHUNK):
        c = counts[k:k + CHUNK].to(torch.int64)
        assert bool((c.sum(1) == n_tot).all()) and bool((c >= 0).all())
        b = ((c[:, 0] - c[:, 1] + n_tot) * n_bins).div(2 * n_tot, rounding_mode="floor")
        ref += torch.bincount(b.clamp(0, n_bins - 1), minlength=n_bins)
        del c, b
    assert int(hist.sum()) == M
    np.testing.assert_array_equal(hist.cpu().numpy(), ref.cpu().numpy())


def test_bitwise_then_lanes_at_2p32_minus_1(torch):
    n_tot = 1024
    net = frank_network(n_tot)
    n = bwg.Network(net)
    sched = (0.25, 0.3125)   # about 128 events per replica, then 32 more
    ranges = ((0, 4096), (PIECE - 64, 128), (3_000_000_007, 40), (M_MAX - 97, 97))
    oracles = [_oracle(net, M_MAX, f, c, sched[:1], ssa.DRAW_EVENT) for f, c in ranges]
    _need(torch, 175 * 10 ** 9)
    _say("case bitwise M = 2^32 - 1")
    ens = bwg.Ensemble(n, M_MAX, seed=0)
    ens.init_fixed((0, 0, n_tot))
    ens.advance(sched[0])
    ev, real = ens.read_events()
    torch.cuda.synchronize()
    # budgets of the first advance, drawn per replica
    q = quantize(net)
    table = poisson_table(q["Lambda"] * sched[0])
    for (first, count), o in zip(ranges, oracles):
        np.testing.assert_array_equal(ev[first:first + count].cpu().numpy().astype(np.uint64),
                                      o.E)
        np.testing.assert_array_equal(o.E, ssa.budgets(0, 0, 0, first, count, table))
    # real events of the first 128 words
    np.testing.assert_array_equal(real[:128].cpu().numpy().astype(np.uint64),
                                  np.add.reduceat(oracles[0].real.astype(np.uint64),
                                                  np.arange(0, 4096, 32)))
    del ev, real
    _say("case lanes after bitwise, M = 2^32 - 1")
    ens.set_engine("lanes")
    ens.advance(sched[1])
    for o in oracles:
        o.advance(sched[1])
    counts = ens.read_counts()
    hist = ens.histogram(256)
    torch.cuda.synchronize()
    for (first, count), o in zip(ranges, oracles):
        np.testing.assert_array_equal(counts[first:first + count].cpu().numpy(), o.counts)
    _check_all(torch, counts, n_tot, hist, 256)
    del counts, hist
    ev, _ = ens.read_events()
    for (first, count), o in zip(ranges, oracles):
        np.testing.assert_array_equal(ev[first:first + count].cpu().numpy().astype(np.uint64),
                                      o.E)
    del ev, ens
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_plain_engine_beyond_2p31_replicas(torch):
    # 3M int32 counts pass 2^33, so their copy takes five dispatches
    n_tot = 1024
    net = frank_network(n_tot)
    M = PIECE + (1 << 30) + 5
    sched = (0.25,)
    ranges = ((0, 2048), (PIECE - 32, 64), (M - 50, 50))
    oracles = [_oracle(net, M, f, c, sched, ssa.DRAW_PLAIN) for f, c in ranges]
    _need(torch, 170 * 10 ** 9)
    _say("case plain M = 2^31 + 2^30 + 5")
    ens = bwg.Ensemble(bwg.Network(net), M, seed=0, engine="plain")
    ens.init_fixed((0, 0, n_tot))
    ens.advance(sched[0])
    sel = [f + c - 1 for f, c in ranges] + [M, M_MAX]
    traj, _ = ens.record([sched[0]], sel)
    counts = ens.read_counts()
    hist = ens.histogram(256)
    torch.cuda.synchronize()
    for (first, count), o in zip(ranges, oracles):
        np.testing.assert_array_equal(counts[first:first + count].cpu().numpy(), o.counts)
    t = traj.cpu().numpy()[0]
    np.testing.assert_array_equal(t[:3], np.stack([o.counts[-1] for o in oracles]))
    assert (t[3:] == -1).all()
    _check_all(torch, counts, n_tot, hist, 256)
    del counts, hist
    ev, real = ens.read_events()
    for (first, count), o in zip(ranges, oracles):
        np.testing.assert_array_equal(ev[first:first + count].cpu().numpy().astype(np.uint64),
                                      o.E)
        np.testing.assert_array_equal(real[first:first + count].cpu().numpy().astype(np.uint64),
                                      o.real)
    del ev, real, ens
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_batch_beyond_2p31_replicas(torch):
    """A persistent batch whose members hold 2.7e9 replicas together: the
    batch's budget launch (one work-item per replica of every member) takes
    two dispatches, the second starting inside the second member.  Sampled
    replicas of each member, including both sides of the boundary, against
    the oracle."""
    mix = [(frank_network(16, k0=0.05), (1 << 30) + 3),
           (frank_network(24, k0=0.02), (1 << 30) + (1 << 29) + 7)]
    t_end = 2.0
    M1 = mix[0][1]
    samples = [((0, 64), (M1 - 40, 40)),
               ((0, 32), (PIECE - M1 - 32, 64), (mix[1][1] - 50, 50))]
    oracles = []
    for k, ((net, M), ranges) in enumerate(zip(mix, samples)):
        row = []
        for first, count in ranges:
            o = ssa.OracleEnsemble(net, M, seed=3, net_id=100 + k, first=first, count=count)
            o.init(("fixed", (0, 0, net["n_tot"])))
            o.advance(t_end)
            row.append(o)
        oracles.append(row)
    _need(torch, 100 * 10 ** 9)
    _say("case batch of", [M for _, M in mix], "replicas")
    ens = []
    for k, (net, M) in enumerate(mix):
        e = bwg.Ensemble(bwg.Network(net), M, seed=3, net_id=100 + k)
        e.init_fixed((0, 0, net["n_tot"]))
        ens.append(e)
    b = bwg.Batch(ens)
    b.advance([t_end, t_end])
    torch.cuda.synchronize()
    for e, ranges, row, (net, M) in zip(ens, samples, oracles, mix):
        counts = e.read_counts()
        ev = e.read_events()[0]
        torch.cuda.synchronize()
        for (first, count), o in zip(ranges, row):
            np.testing.assert_array_equal(counts[first:first + count].cpu().numpy(), o.counts)
            np.testing.assert_array_equal(ev[first:first + count].cpu().numpy().astype(np.uint64),
                                          o.E)
        for k in range(0, M, CHUNK):
            assert bool((counts[k:k + CHUNK].to(torch.int64).sum(1) == net["n_tot"]).all())
        del counts, ev
    del b, ens
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
