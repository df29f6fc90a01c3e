"""Degenerate cases of the chain against the oracle, bit for bit: one and two
molecules per replica (one count plane, bimolecular reactions that can
never fire or fire from one state only), absorbing starts (no reaction has
positive weight, so every event is null and only the event counters move),
and a threshold range of a single plane (the paper's network at N_tot <= 2,
W = 2)."""

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


CASES = [
    # (id, network, replicas, start, schedule)
    ("frank-N1", frank_network(1, k0=0.05), 1000, ("fixed", (0, 0, 1)),
     [("advance", 40.0), ("step", 300)]),
    ("frank-N2", frank_network(2, k0=0.05), 777, ("fixed", (0, 0, 2)),
     [("advance", 7.0), ("step", 500), ("advance", 9.5)]),
    ("frank-N2-LD", frank_network(2, k0=0.05), 333, ("fixed", (1, 1, 0)),
     [("step", 200)]),
    ("paper-N1", paper_network(1), 1000, ("multinomial",), [("advance", 30.0)]),
    ("paper-N2", paper_network(2), 513, ("multinomial",), [("step", 1000), ("advance", 20.0)]),
    # absorbing: all L, nothing can fire
    ("frank-all-L", frank_network(64, k0=0.02), 600, ("fixed", (64, 0, 0)),
     [("advance", 3.0), ("step", 100)]),
    ("paper-all-D", paper_network(32), 300, ("fixed", (0, 32, 0)), [("step", 2000)]),
]


@pytest.mark.parametrize("engine", ["bitwise", "lanes", "plain"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_degenerate_cases_match_oracle(torch, case, engine):
    name, net, M, init, sched = case
    print("case", name, engine, flush=True)
    e = bwg.Ensemble(bwg.Network(net), M, seed=6, net_id=4, engine=engine)
    e.init(init)
    for op, v in sched:
        getattr(e, op)(v)
    counts = e.read_counts().cpu().numpy()
    ev, real = e.read_events()
    ev, real = ev.cpu().numpy().astype(np.uint64), real.cpu().numpy().astype(np.uint64)
    o = ssa.OracleEnsemble(net, M, seed=6, net_id=4,
                           draw=ssa.DRAW_PLAIN if engine == "plain" else ssa.DRAW_EVENT)
    o.init(init)
    for op, v in sched:
        getattr(o, op)(v)
    np.testing.assert_array_equal(counts, o.counts)
    np.testing.assert_array_equal(ev, o.E)
    if engine == "plain":
        np.testing.assert_array_equal(real, o.real)
    else:
        g = np.zeros((M + 31) // 32, dtype=np.uint64)
        np.add.at(g, np.arange(M) // 32, o.real.astype(np.uint64))
        np.testing.assert_array_equal(real, g)
    assert (counts.sum(1) == net["n_tot"]).all()
    if name.endswith(("all-L", "all-D")):
        # absorbing: the start never changes and no event is real
        assert (counts == np.array(init[1])).all() and int(real.sum()) == 0
        assert (ev > 0).all()
