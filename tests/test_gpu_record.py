"""Trajectories of chosen replicas and first passages to homochirality
(bwg_ensemble_record) against the oracle advanced through the same grid."""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from workloads import frank_network, paper_network

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _oracle_record(net, M, seed, net_id, init, grid, sel, threshold, draw):
    o = ssa.OracleEnsemble(net, M, seed=seed, net_id=net_id, draw=draw)
    o.init(init)
    traj = np.zeros((len(grid), len(sel), 3), np.int32)
    first = np.full(M, -1, np.int64)
    for k, t in enumerate(grid):
        o.advance(t)
        for j, i in enumerate(sel):
            traj[k, j] = o.counts[i] if i < M else -1
        d = np.abs(o.counts[:, 0].astype(np.int64) - o.counts[:, 1])
        first[(first < 0) & (d >= threshold)] = k
    return traj, first, o


@pytest.mark.parametrize("engine,shared", [("bitwise", False), ("plain", False),
                                           ("lanes", False), ("bitwise", True)])
def test_record_matches_oracle(torch, engine, shared):
    """The paper's figure setting: its network, multinomial starts around the
    racemic state, L and D of a few replicas over time, and the first grid
    time at which each replica's |N_L - N_D| reaches 3/4 of N."""
    net = paper_network(32)
    M, seed, net_id = 777, 3, 5
    grid = list(np.linspace(0.01, 0.6, 40))
    sel = [0, 5, 31, 32, 500, 776, 777, 10 ** 6]          # the last two are past the end
    draw = ssa.DRAW_SHARED if shared else (ssa.DRAW_PLAIN if engine == "plain" else ssa.DRAW_EVENT)
    e = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=net_id, engine=engine,
                     shared_threshold=shared)
    e.init(("multinomial",))
    traj, first = e.record(grid, sel, threshold=24)
    t_ref, f_ref, o = _oracle_record(net, M, seed, net_id, ("multinomial",), grid, sel, 24, draw)
    np.testing.assert_array_equal(traj.cpu().numpy(), t_ref)
    np.testing.assert_array_equal(first.cpu().numpy(), f_ref)
    np.testing.assert_array_equal(e.read_counts().cpu().numpy(), o.counts)
    assert (t_ref[:, -2:] == -1).all()
    assert (f_ref >= 0).sum() > M // 4          # many replicas reach homochirality


def test_record_continues_and_equals_advances(torch):
    """Two records with a carried first-passage tensor equal one record, and
    the trajectory equals advances with a read after each."""
    net = frank_network(64, k0=0.02)
    M = 3000
    grid = [0.5 * (k + 1) for k in range(12)]
    a = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=1)
    b = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=1)
    c = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=1)
    for x in (a, b, c):
        x.init(("fixed", (0, 0, 64)))
    sel = list(range(0, M, 97))
    ta, fa = a.record(grid, sel, threshold=20)
    tb1, fb = b.record(grid[:5], sel, threshold=20)
    tb2, fb = b.record(grid[5:], sel, threshold=20, first=fb)
    np.testing.assert_array_equal(ta.cpu().numpy(), np.concatenate([tb1.cpu().numpy(),
                                                                     tb2.cpu().numpy()]))
    fb = fb.cpu().numpy()
    fb[fb >= 0] += 0
    fa = fa.cpu().numpy()
    # the second record counts its grid points from 0
    second = (fa >= 5)
    np.testing.assert_array_equal(fa[~second], fb[~second])
    np.testing.assert_array_equal(fa[second] - 5, fb[second])
    for k, t in enumerate(grid):
        c.advance(t)
        np.testing.assert_array_equal(ta[k].cpu().numpy(), c.read_counts().cpu().numpy()[sel])


def test_record_rejects_bad_grids(torch):
    e = bwg.Ensemble(bwg.Network(frank_network(32)), 64)
    e.init(("fixed", (0, 0, 32)))
    e.advance(1.0)
    with pytest.raises(bwg.BwgError):
        e.record([0.5, 2.0], [0])                  # before t_now
    with pytest.raises(bwg.BwgError):
        e.record([2.0, 1.5], [0])                  # decreasing
    lat = bwg.Ensemble(bwg.Network(frank_network(12, lx=4, ly=4, hop=0.1, site_planes=4)), 64)
    lat.init(("uniform_site", 9, 15))
    with pytest.raises(bwg.BwgError):
        lat.record([1.0], [0])
    out, first = e.record([], [0])                 # empty grid: nothing to do
    assert out.shape == (0, 1, 3) and first is None
