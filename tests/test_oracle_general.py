"""Pins of the oracle on general networks: species counts other than 3 and
open networks (molecule count not conserved, every count capped at n_tot, a
firing past the cap does nothing).  Every check is against something other
than the oracle: closed-form laws of pure death and pure birth, the exact
master equation of the truncated chain, brute-force bounds of the total
weight, and the Python direct method for the C one."""

import math

import numpy as np
import pytest

from oracle import master, ssa
from oracle.quantize import quantize, weights, state_change
from test_oracle_pins import chi2_pvalue, _empirical


def net_of(species, reactions, rates, n_tot, open_net=False):
    return {"species": tuple(species), "reactants": [r for r, _ in reactions],
            "products": [p for _, p in reactions], "rates": [float(k) for k in rates],
            "n_tot": int(n_tot), "lx": 0, "ly": 0, "hop_rates": [0.0] * len(species),
            "site_planes": 0, "exact_integer": False, "open": open_net}


def death(n0=20, k=0.3):
    return net_of("A", [((1,), (0,))], [k], n0, open_net=True)


def birth(cap=30, k=0.5):
    return net_of("A", [((1,), (2,))], [k], cap, open_net=True)


def lotka_volterra(cap=12):
    # X -> 2X, X + Y -> 2Y, Y -> 0
    return net_of("XY", [((1, 0), (2, 0)), ((1, 1), (0, 2)), ((0, 1), (0, 0))],
                  [1.0, 0.1, 0.6], cap, open_net=True)


def cycle4(n=8):
    # A + B -> 2B, B + C -> 2C, C -> D, D -> A (closed, 4 species)
    return net_of("ABCD", [((1, 1, 0, 0), (0, 2, 0, 0)), ((0, 1, 1, 0), (0, 0, 2, 0)),
                           ((0, 0, 1, 0), (0, 0, 0, 1)), ((0, 0, 0, 1), (1, 0, 0, 0))],
                  [0.2, 0.15, 0.5, 0.3], n)


def dimer2(n=10):
    # 2X -> X + Y, Y -> X (closed, 2 species)
    return net_of("XY", [((2, 0), (1, 1)), ((0, 1), (1, 0))], [0.1, 0.4], n)


def run(net, M, start, sched, seed, draw=ssa.DRAW_EVENT):
    E = ssa.OracleEnsemble(net, M, seed=seed, net_id=3, draw=draw)
    E.init(("fixed", start))
    for op, v in sched:
        getattr(E, op)(v)
    return E


@pytest.mark.parametrize("draw", [ssa.DRAW_EVENT, ssa.DRAW_PLAIN])
def test_pure_death_is_binomial(oracle_lib, draw):
    # each molecule dies independently at the quantised rate c / s:
    # N(t) ~ Binomial(N0, exp(-k t))
    net = death()
    q = quantize(net)
    k = q["c"][0] / q["s"]
    E = run(net, 8192, (20,), [("advance", 1.5), ("advance", 3.0)], seed=21, draw=draw)
    p = math.exp(-k * 3.0)
    st = [(n,) for n in range(21)]
    probs = np.array([math.comb(20, n) * p ** n * (1 - p) ** (20 - n) for n in range(21)])
    assert chi2_pvalue(_empirical(E.counts, st), probs * 8192) > 1e-4


def test_pure_birth_is_geometric_with_the_cap(oracle_lib):
    # Yule process from one molecule: P(N = n) = p (1 - p)^(n - 1), p =
    # exp(-k t), for n below the cap; the cap blocks every further birth, so
    # it holds the rest of the mass
    cap = 30
    net = birth(cap)
    q = quantize(net)
    k = q["c"][0] / q["s"]
    E = run(net, 8192, (1,), [("advance", 4.0)], seed=22)
    assert (E.counts <= cap).all() and (E.counts >= 1).all()
    p = math.exp(-k * 4.0)
    probs = np.array([p * (1 - p) ** (n - 1) for n in range(1, cap)] + [(1 - p) ** (cap - 1)])
    st = [(n,) for n in range(1, cap + 1)]
    assert chi2_pvalue(_empirical(E.counts, st), probs * 8192) > 1e-4
    assert (E.counts == cap).sum() > 100      # the cap is really reached


def test_open_two_species_network_matches_master_equation(oracle_lib):
    net = lotka_volterra()
    q = quantize(net)
    K = 200
    E = run(net, 16384, (5, 3), [("step", 120), ("step", 80)], seed=23)
    st, probs = master.fixed_k_probs(net, q, (5, 3), K)
    assert abs(probs.sum() - 1) < 1e-12
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4
    assert (E.counts.max(0) == 12).any()      # the cap takes part


def test_open_network_time_law(oracle_lib):
    net = lotka_volterra(10)
    q = quantize(net)
    E = run(net, 16384, (4, 2), [("advance", 1.0), ("advance", 2.5)], seed=24)
    st, probs = master.time_probs(net, q, {(4, 2): 1.0}, 2.5)
    assert abs(probs.sum() - 1) < 1e-9
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


@pytest.mark.parametrize("make,start", [(cycle4, (3, 2, 2, 1)), (dimer2, (10, 0))])
def test_closed_networks_of_other_species_counts(oracle_lib, make, start):
    net = make()
    q = quantize(net)
    E = run(net, 16384, start, [("step", 150)], seed=25)
    assert (E.counts.sum(1) == net["n_tot"]).all()
    st, probs = master.fixed_k_probs(net, q, start, 150)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4
    E = run(net, 16384, start, [("advance", 2.0)], seed=26)
    st, probs = master.time_probs(net, q, {tuple(start): 1.0}, 2.0)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


@pytest.mark.parametrize("make", [death, birth, lotka_volterra, cycle4, dimer2])
def test_weight_bound_covers_every_state(make):
    # the uniformisation bound W = 2^B is at or above the total weight of
    # every state of the state space (brute force)
    net = make()
    q = quantize(net)
    S = len(net["species"])
    best = max(sum(weights(net, q, s))
               for s in master.states(net["n_tot"], S, bool(net.get("open"))))
    assert best <= q["max_total"] <= q["W"]
    if net.get("open"):   # attained at the corner of the box
        assert best == q["max_total"]


@pytest.mark.parametrize("make,start", [(lotka_volterra, (5, 3)), (birth, (1,)),
                                        (cycle4, (3, 2, 2, 1)), (dimer2, (10, 0))])
@pytest.mark.parametrize("draw", [ssa.DRAW_EVENT, ssa.DRAW_PLAIN])
def test_c_oracle_matches_python_direct_method(oracle_lib, make, start, draw):
    net = make()
    q = quantize(net)
    n = 24
    counts = np.tile(np.array(start, np.int32), (n, 1))
    E0 = np.arange(n, dtype=np.uint64) * 5
    K = np.full(n, 90, dtype=np.uint64)
    out, real, _ = ssa.run_events(net, q, 6, 4, 40, counts, E0, K, draw=draw)
    nu = state_change(net)
    for k in range(n):
        N, picked = ssa.py_events(net, q, 6, 4, 40 + k, list(start), int(E0[k]), 90, draw=draw)
        assert list(out[k]) == N
        assert int(real[k]) == sum(1 for r in picked if r >= 0 and any(nu[r]))


def test_open_network_refuses_counts_above_the_cap(oracle_lib):
    with pytest.raises(ValueError):
        ssa.OracleEnsemble(lotka_volterra(), 4).init(("fixed", (13, 0)))
    with pytest.raises(ValueError):
        quantize({**lotka_volterra(), "open": False})   # not count-conserving


# ---- weights beyond 32 threshold planes (fixed-point rates at higher precision)

def frank_fine(n_tot=10, k0=0.0137, bits=26):
    """The Frank network with k1 = k2 = 1/N_tot quantised to 26 bits of
    precision: c = (7.4e7, 7.4e7, 2^29, 2^29, 2^29), W = 2^35."""
    from workloads import frank_network
    net = frank_network(n_tot, k0=k0)
    return net, quantize(net, precision_bits=bits)


def test_wide_thresholds_follow_the_master_equation(oracle_lib):
    # 35 threshold planes: every event draws 9 Philox quads per word and
    # compares a 35-bit n; dropping the planes above 32 would make reactions
    # 8 times likelier and fail both laws
    net, q = frank_fine()
    assert q["B"] == 35 and max(q["c"]) < (1 << 32)
    start = (0, 0, 10)
    E = ssa.OracleEnsemble(net, 16384, seed=31, net_id=7, q=q)
    E.init(("fixed", start))
    E.step(400)
    st, probs = master.fixed_k_probs(net, q, start, 400)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4
    E = ssa.OracleEnsemble(net, 16384, seed=32, net_id=7, q=q)
    E.init(("fixed", start))
    E.advance(0.6)
    st, probs = master.time_probs(net, q, {start: 1.0}, 0.6)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


def test_wide_thresholds_c_oracle_matches_python_direct_method(oracle_lib):
    net, q = frank_fine(12)
    n = 16
    counts = np.tile(np.array((2, 3, 7), np.int32), (n, 1))
    E0 = np.arange(n, dtype=np.uint64) * 11
    K = np.full(n, 120, dtype=np.uint64)
    out, real, _ = ssa.run_events(net, q, 9, 5, 70, counts, E0, K)
    nu = state_change(net)
    for k in range(n):
        N, picked = ssa.py_events(net, q, 9, 5, 70 + k, [2, 3, 7], int(E0[k]), 120)
        assert list(out[k]) == N
        assert int(real[k]) == sum(1 for r in picked if r >= 0 and any(nu[r]))


def test_plain_draw_refuses_wide_thresholds(oracle_lib):
    net, q = frank_fine()
    with pytest.raises(ValueError):
        ssa.run_events(net, q, 1, 1, 0, np.zeros((4, 3), np.int32) + [0, 0, 10],
                       np.zeros(4, np.uint64), np.ones(4, np.uint64), draw=ssa.DRAW_PLAIN)
    with pytest.raises(ValueError):
        ssa.py_events(net, q, 1, 1, 0, [0, 0, 10], 0, 1, draw=ssa.DRAW_PLAIN)
