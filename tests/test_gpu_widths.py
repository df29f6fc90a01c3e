"""Word widths of the bit-sliced engine: 16, 32 or 64 replicas per thread.
Every draw is keyed by the 32-lane word and the lane, so the results are the
same at every width: each width is compared with the oracle on small cases
(ragged replica counts: an odd number of words for 64, half-filled halves
for 16) and with the 32-replica word at full size; per-replica and shared
thresholds, advances, fixed steps and capped launches."""

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from oracle import ssa
from workloads import config, frank_network, paper_network

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def run(torch, net, M, init, sched, wb, shared=False, epl=0, seed=5, net_id=2):
    print("width case", wb, net["n_tot"], M, init, sched, shared, epl, flush=True)
    e = bwg.Ensemble(bwg.Network(net), M, seed=seed, net_id=net_id, word_bits=wb,
                     shared_threshold=shared, events_per_launch=epl)
    e.init(init)
    for op, v in sched:
        getattr(e, op)(v)
    ev, real = e.read_events()
    out = (e.read_counts().cpu().numpy(), ev.cpu().numpy().astype(np.uint64),
           real.cpu().numpy().astype(np.uint64))
    torch.cuda.synchronize()
    return out


CASES = [
    (lambda: frank_network(32), 2048 + 17, ("fixed", (0, 0, 32)), [("advance", 20.0)], False, 0),
    (lambda: frank_network(1024), 333, ("fixed", (0, 0, 1024)), [("advance", 0.3), ("step", 77)],
     False, 0),
    (lambda: paper_network(48), 1000, ("multinomial",), [("step", 1500), ("step", 33)], False, 400),
    (lambda: paper_network(100), 97, ("multinomial",), [("step", 2000)], True, 0),
    (lambda: paper_network(24), 65, ("multinomial",), [("advance", 6.0), ("advance", 9.0)], True, 0),
]


@pytest.mark.parametrize("wb", [16, 64])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_widths_match_oracle(torch, wb, case):
    make, M, init, sched, shared, epl = CASES[case]
    net = make()
    counts, ev, real = run(torch, net, M, init, sched, wb, shared, epl)
    o = ssa.OracleEnsemble(net, M, seed=5, net_id=2,
                           draw=ssa.DRAW_SHARED if shared else ssa.DRAW_EVENT)
    o.init(init)
    for op, v in sched:
        getattr(o, op)(v)
    np.testing.assert_array_equal(counts, o.counts)
    np.testing.assert_array_equal(ev, o.E)
    g = np.zeros((M + 31) // 32, dtype=np.uint64)
    np.add.at(g, np.arange(M) // 32, o.real.astype(np.uint64))
    np.testing.assert_array_equal(real, g)


@pytest.mark.parametrize("wb", [16, 64])
def test_widths_equal_32_at_full_size(torch, wb):
    c = config("c1")
    sched = [("advance", 2.0), ("step", 100)]
    a = run(torch, c["net"], c["replicas"], c["init"], sched, 32, seed=0, net_id=0)
    b = run(torch, c["net"], c["replicas"], c["init"], sched, wb, seed=0, net_id=0)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    net = paper_network(1024)
    M = (1 << 22) + 33
    a = run(torch, net, M, ("multinomial",), [("step", 300)], 32, shared=True, seed=3, net_id=1)
    b = run(torch, net, M, ("multinomial",), [("step", 300)], wb, shared=True, seed=3, net_id=1)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_width_refusals(torch):
    n = bwg.Network(frank_network(300, k0=0.002))   # run-time weights only
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(n, 100, word_bits=64)
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(bwg.Network(frank_network(32)), 100, word_bits=48)
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble(bwg.Network(frank_network(32)), 100, word_bits=16, engine="plain")
