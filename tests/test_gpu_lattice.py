"""Parity of the HIP lattice path with the CPU lattice oracle: every replica's
site counts bit for bit, on small lattices (all replicas, ragged words, two
component groups, degenerate one-site-wide axes) and on the 64 x 64 lattice
of 2^16 replicas (sampled replicas, in the launch configuration bench.py
times)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2412_16613_amd as bwg  # noqa: E402
from oracle.lattice import OracleLattice  # noqa: E402
from workloads import config, frank_network  # noqa: E402

pytestmark = pytest.mark.gpu

UNIFORM = ("uniform_site", 9, 15)


def lattice(side_x, side_y, **kw):
    kw.setdefault("hop", 0.1)
    kw.setdefault("site_planes", 4)
    return frank_network(12, lx=side_x, ly=side_y, **kw)


def pair(net, M, seed=1, net_id=5, init=UNIFORM, first=0, count=None, stride=1,
         lds_stage=True):
    ens = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=net_id, lds_stage=lds_stage)
    ens.init(init)
    orc = OracleLattice(net, M, seed=seed, net_id=net_id, first=first, count=count,
                        stride=stride, threads=8)
    orc.init(init)
    return ens, orc


def gpu_sites(ens, orc):
    if orc.stride == 1:
        return ens.read_sites(orc.first, orc.n).cpu().numpy()
    return np.stack([ens.read_sites(orc.first + k * orc.stride, 1).cpu().numpy()[0]
                     for k in range(orc.n)])


def check(ens, orc, what=""):
    torch.cuda.synchronize()
    g = gpu_sites(ens, orc)
    bad = np.nonzero((g != orc.sites).any(axis=(1, 2)))[0]
    assert len(bad) == 0, "%s: %d replicas differ, first %s" % (what, len(bad), bad[:8])


def test_init_uniform_site_matches_oracle():
    ens, orc = pair(lattice(8, 8), 3000)
    check(ens, orc, "init")
    assert (orc.sites[:, :, 2] >= 9).all()


@pytest.mark.parametrize("lx,ly,M,K", [(4, 4, 100, 3000), (8, 8, 2048 + 70, 2500),
                                       (5, 3, 33, 4000), (2, 2, 64, 20000),
                                       (1, 4, 40, 5000), (3, 1, 31, 5000),
                                       (1, 1, 100, 3000), (2, 1, 65, 4000)])
def test_fixed_event_count(lx, ly, M, K):
    # (1, 1): a single site, every hop leads back to it; (2, 1): both
    # x-directions lead to the same neighbour
    ens, orc = pair(lattice(lx, ly), M)
    ens.step(K)
    orc.step(K)
    check(ens, orc, "step")
    torch.cuda.synchronize()
    blocked = ens.read_blocked().cpu().numpy().astype(np.uint64)
    g = np.zeros((M + 31) // 32, dtype=np.uint64)
    np.add.at(g, np.arange(M) // 32, orc.blocked.astype(np.uint64))
    np.testing.assert_array_equal(blocked, g)


@pytest.mark.parametrize("lds_stage", [True, False])
@pytest.mark.parametrize("M", [16384 + 1000 + 7, 40000 + 5])
def test_sliced_workgroups_every_replica(M, lds_stage):
    """Ensembles of 512 words and more: without staging, 4-word slices per
    workgroup and, beyond 16 groups, several launches over bands of groups;
    staged, one word per workgroup with the whole lattice in LDS.  Ragged last
    slice and group, all replicas compared."""
    net = lattice(4, 4)
    ens, orc = pair(net, M, seed=12, lds_stage=lds_stage)
    ens.step(1000)
    orc.step(1000)
    check(ens, orc, "8-word slices, step")
    ens.advance(1.0)
    orc.advance(1.0)
    check(ens, orc, "8-word slices, advance")
    _, real = ens.read_events()
    pad = (-M) % 32
    word = lambda v: np.concatenate([v, np.zeros(pad, v.dtype)]).reshape(-1, 32).sum(1)
    assert (real.cpu().numpy() == word(orc.real.astype(np.int64))).all()


def test_two_advances_and_counters():
    net = lattice(8, 8)
    M = 2048 + 70
    ens, orc = pair(net, M, seed=3)
    for t in (0.7, 2.0):
        ens.advance(t)
        orc.advance(t)
        check(ens, orc, "advance to %g" % t)
    ev, real = ens.read_events()
    blocked = ens.read_blocked()
    torch.cuda.synchronize()
    assert (ev.cpu().numpy() == orc.E.astype(np.int64)).all()
    pad = (-M) % 32
    word = lambda v: np.concatenate([v, np.zeros(pad, v.dtype)]).reshape(-1, 32).sum(1)
    assert (real.cpu().numpy() == word(orc.real.astype(np.int64))).all()
    assert (blocked.cpu().numpy() == word(orc.blocked.astype(np.int64))).all()
    assert orc.blocked.sum() > 0
    tot = ens.read_counts().cpu().numpy()
    assert (tot == orc.totals()).all()
    h = ens.histogram(256).cpu().numpy()
    assert (h == orc.histogram(256).astype(np.int64)).all()


def test_capped_passes_equal_one_advance():
    net = lattice(6, 6)
    M = 300
    a, orc = pair(net, M, seed=9)
    b = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=5)
    b.init(UNIFORM)
    a.advance(40.0)
    b.schedule(40.0)
    passes = 0
    while b.pending():
        b.run(8192)
        passes += 1
    assert passes > 2
    orc.advance(40.0)
    check(a, orc, "advance")
    check(b, orc, "capped passes")
    with pytest.raises(bwg.BwgError):
        b.schedule(41.0)
        b.schedule(42.0)


def test_pure_diffusion_and_fixed_sites():
    net = lattice(7, 5, k0=0.0, k1=0.0, k2=0.0)
    rng = np.random.default_rng(2)
    sites = np.zeros((35, 3), np.int32)
    sites[:, 0] = rng.integers(0, 6, 35)
    sites[:, 1] = rng.integers(0, 5, 35)
    sites[:, 2] = rng.integers(0, 5, 35)
    ens, orc = pair(net, 77, seed=4, init=("sites", sites))
    ens.advance(5.0)
    orc.advance(5.0)
    check(ens, orc, "diffusion")
    assert (orc.totals() == sites.sum(0)).all()


def test_other_rates_take_the_run_time_kernel():
    net = lattice(6, 4, k0=0.03, k1=0.2, k2=0.05, hop=0.37)
    n = bwg.Network(net)
    assert n.quantized()["c"][0] != 246
    ens, orc = pair(net, 130, seed=6, init=("fixed_site", (3, 2, 5)))
    ens.advance(1.5)
    orc.advance(1.5)
    check(ens, orc, "run-time weights")


def test_errors():
    net = lattice(4, 4)
    ens = bwg.Ensemble(bwg.Network(net), 64)
    with pytest.raises(bwg.BwgError):
        ens.init(("uniform_site", 9, 16))
    with pytest.raises(bwg.BwgError):
        ens.init(("fixed_site", (8, 8, 0)))
    with pytest.raises(bwg.BwgError):
        ens.advance(1.0)            # not initialised
    ens.init(UNIFORM)
    with pytest.raises(bwg.BwgError):
        ens.read_sites(60, 10)
    with pytest.raises(bwg.BwgError):
        bwg.Batch([ens])


def test_full_lattice_short_horizon_sampled():
    c = config("c2")
    M = c["replicas"]
    ens, orc = pair(c["net"], M, seed=c["seed"], net_id=c["net_id"], init=c["init"],
                    first=5, count=16, stride=4093)
    ens.advance(0.5)
    orc.advance(0.5)
    check(ens, orc, "64x64, t=0.5")


def test_full_lattice_bench_configuration_sampled():
    """The bench workload: init + advance to t_end = 20 on 2^16 replicas.
    64 replicas one every 1024 (two from each of the 32 component groups,
    both launch bands of 16 groups, different words and lanes) and the last
    two replicas are checked site by site, with their event counts."""
    c = config("c2")
    M = c["replicas"]
    ens = bwg.Ensemble(bwg.Network(c["net"]), M, seed=c["seed"], net_id=c["net_id"])
    ens.init(c["init"]).advance(c["t_end"])
    ev = ens.read_events()[0].cpu().numpy().astype(np.uint64)
    for first, count, stride in ((5, 64, 1024), (M - 2, 2, 1)):
        o = OracleLattice(c["net"], M, seed=c["seed"], net_id=c["net_id"], first=first,
                          count=count, stride=stride, threads=16)
        o.init(c["init"])
        o.advance(c["t_end"])
        check(ens, o, "64x64, t=20, replicas %d + k * %d" % (first, stride))
        np.testing.assert_array_equal(ev[first::stride][:count], o.E)


@pytest.mark.parametrize("lx,ly,kw,M,t", [
    (64, 64, {}, 16384 + 37, 1.0),       # sites 840.. stay in memory, ragged last slice
    (24, 24, {}, 20000, 2.0),            # every site in LDS
    (29, 29, {}, 16384 + 5, 1.0),        # one site (840) beyond the staged ones
    (59, 61, {}, 64 * 600, 0.2)])        # several launch bands
def test_lds_staged_kernel_equals_memory_kernel(lx, ly, kw, M, t):
    """The event kernel that keeps the first 840 sites of each word of a
    4-word slice in LDS gives every replica's site counts, event counts and
    blocked hops of the kernel that keeps them in memory, bit for bit (all
    replicas; ensembles of 512 words and more take the staged kernel)."""
    net = bwg.Network(lattice(lx, ly, **kw))
    out = []
    for stage in (True, False):
        e = bwg.Ensemble(net, M, seed=21, net_id=9, lds_stage=stage)
        e.init(UNIFORM).advance(t)
        ev, real = e.read_events()
        out.append((e.read_sites(0, M), ev, real, e.read_blocked()))
        del e
    for a, b in zip(*out):
        assert torch.equal(a, b)
