"""Networks of other than 3 species and open networks (molecule count not
conserved, every count capped at n_tot) on the bit-sliced kernel compiled
for each network, against the oracle bit for bit: counts of every replica,
events per replica and real events per word; both word-loop forms (the
producer/consumer form up to 32768 words, one wave per word above)."""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from workloads import open_network, random_wide_network

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


def check(torch, net, M, start, sched, seed=3, net_id=7, sample=None):
    print("wide case", len(net["species"]), net.get("open"), net["n_tot"], len(net["rates"]), M,
          start, sched, flush=True)
    e = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=net_id)
    e.init_fixed(start)
    for op, v in sched:
        getattr(e, op)(v)
    counts = e.read_counts().cpu().numpy()
    ev, real = e.read_events()
    ev = ev.cpu().numpy().astype(np.uint64)
    torch.cuda.synchronize()
    assert counts.shape == (M, len(net["species"]))
    if net.get("open"):
        assert (counts >= 0).all() and (counts <= net["n_tot"]).all()
    else:
        assert (counts.sum(1) == net["n_tot"]).all()
    blocks = [(0, M)] if sample is None else sample
    for first, count in blocks:
        o = ssa.OracleEnsemble(net, M, seed=seed, net_id=net_id, first=first, count=count)
        o.init(("fixed", start))
        for op, v in sched:
            getattr(o, op)(v)
        np.testing.assert_array_equal(counts[first:first + count], o.counts)
        np.testing.assert_array_equal(ev[first:first + count], o.E)
        if sample is None:
            np.testing.assert_array_equal(real.cpu().numpy().astype(np.uint64),
                                          _group_sums(o.real, M))
    return counts


@pytest.mark.parametrize("name,cap,start,M", [
    ("death", 20, (20,), 1000), ("birth", 30, (1,), 4096 + 5), ("lotka_volterra", 12, (5, 3), 777),
    ("lotka_volterra", 100, (40, 20), 2048), ("birth", 1000, (3,), 300),
])
def test_open_networks_match_oracle(torch, name, cap, start, M):
    net = open_network(name, cap)
    q = bwg.Network(net).quantized()
    dt = 300.0 / q["Lambda"]
    counts = check(torch, net, M, start, [("advance", dt), ("step", 111), ("advance", 2.5 * dt)])
    if name == "birth" and cap == 30:
        assert (counts == cap).any()          # the cap blocked births


@pytest.mark.parametrize("seed,S,n_tot,R,open_net,M", [
    (0, 4, 8, 5, False, 1000), (1, 2, 10, 6, True, 500), (2, 8, 6, 10, False, 333),
    (3, 5, 20, 8, True, 2048 + 31), (4, 1, 40, 3, True, 64), (5, 3, 30, 6, True, 1024),
    (6, 6, 12, 16, True, 97), (7, 2, 200, 7, False, 700),
])
def test_random_wide_networks_match_oracle(torch, seed, S, n_tot, R, open_net, M):
    net = random_wide_network(seed, S, n_tot, R, open_net)
    q = bwg.Network(net).quantized()
    assert q["gpu_ok"]
    dt = 250.0 / q["Lambda"]
    rng = np.random.default_rng(seed)
    if open_net:
        start = tuple(int(v) for v in rng.integers(0, n_tot // 2 + 1, S))
    else:
        cut = np.sort(rng.integers(0, n_tot + 1, S - 1))
        start = tuple(int(v) for v in np.diff(np.concatenate([[0], cut, [n_tot]])))
    check(torch, net, M, start, [("advance", dt), ("step", 77)], seed=seed, net_id=seed + 40)


def test_one_wave_per_word_form_sampled(torch):
    # more than 32768 words: the compiled kernel's one-wave-per-word form
    net = open_network("lotka_volterra", 60)
    q = bwg.Network(net).quantized()
    M = (1 << 20) + 77
    check(torch, net, M, (20, 10), [("advance", 200.0 / q["Lambda"])],
          sample=[(0, 256), (M // 2 + 3, 64), (M - 77, 77)])


def test_refusals(torch):
    net = bwg.Network(open_network("lotka_volterra", 12))
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(net, 100, engine="plain")
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(net, 100, jit=False)        # only its compiled kernel runs it
    e = bwg.Ensemble(net, 100)
    with pytest.raises(bwg.BwgError):
        e.init_fixed((13, 0))                     # above the cap
    with pytest.raises(bwg.BwgError):
        e.init(("multinomial",))
    e.init_fixed((12, 12))
    with pytest.raises(bwg.BwgError):
        e.histogram(16)
    with pytest.raises(bwg.BwgError):
        bwg.Batch([e])
    e.step(10)                                    # still usable after the refusals
    assert (e.read_events()[0].cpu().numpy() == 10).all()
