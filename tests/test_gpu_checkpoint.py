"""Checkpoint and resume (bwg_ensemble_save / bwg_ensemble_restore).

A run saved between advances and resumed in another ensemble equals the
uninterrupted run bit for bit, and both equal the oracle, on every state
kind (bit planes under both engines, plain counts, lattices) and in the
shared-threshold mode.  A checkpoint whose event counters were set near
2^34 checks the draw contract where the event index leaves 32 bits: the
EVENT and lattice component draws carry bits 32..47 of the event index in
the counter's second word, the PLAIN draw bits 32..47 of event / 4.
"""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from paper_2412_16613_amd import _abi
from oracle import ssa
from oracle.lattice import OracleLattice
from workloads import frank_network, paper_network, random_network

pytestmark = pytest.mark.gpu

MAGIC = 0x31544B5043475742
REG_E, REG_ET = 3, 4
HIGH = (1 << 34) - 7


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _say(*a):
    print(*a, flush=True)


def regions(blob):
    h = np.frombuffer(blob, dtype=np.uint64, count=32)
    assert int(h[0]) == MAGIC and int(h[1]) == 256 and int(h[2]) == len(blob)
    return {int(h[12 + 3 * k]): (int(h[13 + 3 * k]), int(h[14 + 3 * k]))
            for k in range(int(h[11]))}


def u64_region(blob, rid):
    off, nbytes = regions(blob)[rid]
    return np.frombuffer(blob, dtype=np.uint64, count=nbytes // 8, offset=off)


def state(torch, ens):
    ev, real = ens.read_events()
    out = (ens.read_counts().cpu().numpy(), ev.cpu().numpy(), real.cpu().numpy())
    torch.cuda.synchronize()
    return out


def run(ens_or_orc, schedule):
    for op, v in schedule:
        getattr(ens_or_orc, op)(v)


WELL_MIXED = [
    # (id, network, M, init, engine, shared, draw)
    ("frank64-bitwise", frank_network(64, k0=0.02), 1000 + 37, ("fixed", (0, 0, 64)),
     "bitwise", False, ssa.DRAW_EVENT),
    ("paper32-lanes", paper_network(32), 777, ("multinomial",), "lanes", False, ssa.DRAW_EVENT),
    ("frank100-plain", frank_network(100, k0=0.03), 513, ("fixed", (10, 10, 80)), "plain",
     False, ssa.DRAW_PLAIN),
    ("paper32-shared", paper_network(32), 300, ("multinomial",), "bitwise", True,
     ssa.DRAW_SHARED),
    ("general", random_network(3, 50, 6), 640 + 5, ("fixed", (20, 20, 10)), "bitwise", False,
     ssa.DRAW_EVENT),
]


@pytest.mark.parametrize("case", WELL_MIXED, ids=[c[0] for c in WELL_MIXED])
def test_resume_equals_uninterrupted_run(torch, case):
    name, net, M, init, engine, shared, draw = case
    _say("case", name)
    before = [("advance", 0.7), ("step", 150)]
    after = [("advance", 1.9), ("step", 61), ("advance", 2.5)]
    n = bwg.Network(net)
    a = bwg.Ensemble(n, M, seed=4, net_id=2, engine=engine, shared_threshold=shared)
    a.init(init)
    run(a, before)
    blob = a.save()
    run(a, after)
    ref = state(torch, a)
    o = ssa.OracleEnsemble(net, M, seed=4, net_id=2, draw=draw)
    o.init(init)
    run(o, before + after)
    np.testing.assert_array_equal(ref[0], o.counts)
    np.testing.assert_array_equal(ref[1].astype(np.uint64), o.E)
    # restored into a fresh ensemble of the same network (a second handle of
    # an equal network), and for bit planes under the other engine too
    engines = [engine] + ({"bitwise": ["lanes"], "lanes": ["bitwise"]}.get(engine, [])
                          if not shared and name != "general" else [])
    for eng in engines:
        b = bwg.Ensemble(bwg.Network(net), M, seed=4, net_id=2, engine=eng,
                         shared_threshold=shared)
        b.restore(blob)
        run(b, after)
        got = state(torch, b)
        for x, y in zip(got, ref):
            np.testing.assert_array_equal(x, y)
        st = b.stats()
        assert st["advance_index"] == 3 and st["t_now"] == 2.5


def test_resume_with_another_seed_continues_the_saved_state(torch):
    """Other seed and net_id: the saved counts and counters, new draws -- the
    oracle started from the saved state with the new key."""
    net = frank_network(64, k0=0.02)
    M = 500
    a = bwg.Ensemble(bwg.Network(net), M, seed=1, net_id=0)
    a.init_fixed((0, 0, 64))
    a.advance(0.5)
    blob = a.save()
    counts0, ev0, _ = state(torch, a)
    b = bwg.Ensemble(bwg.Network(net), M, seed=9, net_id=3).restore(blob)
    b.advance(1.25)
    counts, ev, _ = state(torch, b)
    o = ssa.OracleEnsemble(net, M, seed=9, net_id=3)
    o.counts, o.E = counts0.copy(), ev0.astype(np.uint64)
    o.t_now, o.advance_index = 0.5, 1
    o.advance(1.25)
    np.testing.assert_array_equal(counts, o.counts)
    np.testing.assert_array_equal(ev.astype(np.uint64), o.E)
    a.advance(1.25)
    assert (a.read_counts().cpu().numpy() != counts).any()


def _lattice_net(lx, ly):
    return frank_network(12, lx=lx, ly=ly, hop=0.1, site_planes=4)


@pytest.mark.parametrize("lx,ly,M", [(4, 4, 300), (8, 8, 16384 + 45)])
def test_lattice_resume_equals_uninterrupted_run(torch, lx, ly, M):
    _say("case lattice", lx, ly, M)
    net = _lattice_net(lx, ly)
    init = ("uniform_site", 9, 15)
    a = bwg.Ensemble(bwg.Network(net), M, seed=3, net_id=1)
    a.init(init)
    a.advance(0.4)
    blob = a.save()
    a.advance(0.9)
    a.step(500)
    b = bwg.Ensemble(bwg.Network(net), M, seed=3, net_id=1, lds_stage=False).restore(blob)
    b.advance(0.9)
    b.step(500)
    torch.cuda.synchronize()
    sa, sb = a.read_sites().cpu().numpy(), b.read_sites().cpu().numpy()
    np.testing.assert_array_equal(sa, sb)
    for x, y in zip(a.read_events(), b.read_events()):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    np.testing.assert_array_equal(a.read_blocked().cpu().numpy(),
                                  b.read_blocked().cpu().numpy())
    o = OracleLattice(net, M, seed=3, net_id=1, count=min(M, 300), threads=8)
    o.init(init)
    o.advance(0.4)
    o.advance(0.9)
    o.step(500)
    np.testing.assert_array_equal(sb[:o.n], o.sites)


HIGH_CASES = [
    ("bitwise", frank_network(64, k0=0.02), ("fixed", (0, 0, 64)), ssa.DRAW_EVENT),
    ("lanes", paper_network(32), ("multinomial",), ssa.DRAW_EVENT),
    ("plain", frank_network(100, k0=0.03), ("fixed", (10, 10, 80)), ssa.DRAW_PLAIN),
]


@pytest.mark.parametrize("case", HIGH_CASES, ids=[c[0] for c in HIGH_CASES])
def test_event_indices_beyond_32_bits(torch, case):
    """Replicas restored at events 2^34 - 7 - (i mod 11) run 40 more: the
    event index crosses 2^34 (bits 32..47 of the index, and for the PLAIN
    draw of index / 4, change) and must match the oracle from the same
    counters."""
    engine, net, init, draw = case
    M = 1000 + 19
    _say("case high events", engine)
    a = bwg.Ensemble(bwg.Network(net), M, seed=7, net_id=1, engine=engine)
    a.init(init)
    blob = a.save()
    E0 = (HIGH - (np.arange(M) % 11)).astype(np.uint64)
    for rid in (REG_E, REG_ET):
        u64_region(blob, rid)[:M] = E0
    a.restore(blob)
    a.step(40)
    counts, ev, _ = state(torch, a)
    o = ssa.OracleEnsemble(net, M, seed=7, net_id=1, draw=draw)
    o.init(init)
    o.E = E0.copy()
    o.step(40)
    np.testing.assert_array_equal(counts, o.counts)
    np.testing.assert_array_equal(ev.astype(np.uint64), o.E)
    assert (o.E > (1 << 34)).all() and (E0 < (1 << 34)).all()


def test_lattice_event_indices_beyond_32_bits(torch):
    net = _lattice_net(4, 4)
    M = 200
    init = ("uniform_site", 9, 15)
    a = bwg.Ensemble(bwg.Network(net), M, seed=2, net_id=6)
    a.init(init)
    blob = a.save()
    E0 = (HIGH - (np.arange(M) % 11)).astype(np.uint64)
    for rid in (REG_E, REG_ET):
        u64_region(blob, rid)[:M] = E0
    a.restore(blob)
    a.step(300)
    torch.cuda.synchronize()
    o = OracleLattice(net, M, seed=2, net_id=6, threads=8)
    o.init(init)
    o.E = E0.copy()
    o.step(300)
    np.testing.assert_array_equal(a.read_sites().cpu().numpy(), o.sites)
    np.testing.assert_array_equal(a.read_events()[0].cpu().numpy().astype(np.uint64), o.E)


def test_checkpoint_errors(torch):
    net = frank_network(64, k0=0.02)
    M = 400
    a = bwg.Ensemble(bwg.Network(net), M, seed=1)
    with pytest.raises(bwg.BwgError) as e:
        a.save()                                   # before init
    assert e.value.code == _abi.BWG_EINVAL
    a.init_fixed((0, 0, 64))
    a.schedule(1.0)
    a.run(5)
    with pytest.raises(bwg.BwgError) as e:
        a.save()                                   # events pending
    assert e.value.code == _abi.BWG_EINVAL
    while a.pending():
        a.run(0)
    blob = a.save()
    good = state(torch, a)

    def refused(target, b, code=_abi.BWG_EINVAL):
        with pytest.raises(bwg.BwgError) as e:
            target.restore(b)
        assert e.value.code == code

    refused(bwg.Ensemble(bwg.Network(net), M + 1), blob)                       # replicas
    refused(bwg.Ensemble(bwg.Network(frank_network(65, k0=0.02)), M), blob)    # network
    refused(bwg.Ensemble(bwg.Network(net), M, engine="plain"), blob)           # state kind
    refused(bwg.Ensemble(bwg.Network(net), M, shared_threshold=True), blob)    # shared mode
    b = bwg.Ensemble(bwg.Network(net), M, seed=1)
    refused(b, blob[:-8])                                                      # truncated
    bad = bytearray(blob)
    bad[0] ^= 1
    refused(b, bad)                                                            # magic
    bad = bytearray(blob)
    u64_region(bad, REG_ET)[3] += 1
    refused(b, bad)                                                            # pending events
    bad = bytearray(blob)
    for rid in (REG_E, REG_ET):
        u64_region(bad, rid)[7] = 1 << 47
    refused(b, bad, _abi.BWG_ERANGE)                                           # event index
    # refusals leave the ensemble untouched; the good checkpoint restores
    b.restore(blob)
    for x, y in zip(state(torch, b), good):
        np.testing.assert_array_equal(x, y)
    sh = bwg.Ensemble(bwg.Network(paper_network(32)), 100, shared_threshold=True)
    sh.init(("multinomial",))
    sblob = sh.save()
    for rid in (REG_E, REG_ET):
        u64_region(sblob, rid)[5] += 1
    refused(bwg.Ensemble(bwg.Network(paper_network(32)), 100, shared_threshold=True), sblob)
