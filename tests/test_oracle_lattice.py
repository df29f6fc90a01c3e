"""Pins of the compartment (lattice) oracle against laws fixed independently
of it: exact finite-state chains written from the reaction and hop rules,
the closed-form random walk of a lone molecule, uniform draws and the
conservation laws.  CPU only."""

import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import lattice, ssa
from oracle.lattice import OracleLattice, quantize_lattice
from workloads import frank_network

G = lattice.GROUP_REPLICAS


@pytest.fixture(scope="module", autouse=True)
def _built():
    ssa.build(force=False)


def chi2_p(observed, expected, min_expected=5.0):
    observed = np.asarray(observed, float)
    expected = np.asarray(expected, float)
    order = np.argsort(expected)
    o_p, e_p, ao, ae = [], [], 0.0, 0.0
    for i in order:
        ao += observed[i]
        ae += expected[i]
        if ae >= min_expected:
            o_p.append(ao)
            e_p.append(ae)
            ao = ae = 0.0
    if ae > 0 and e_p:
        o_p[-1] += ao
        e_p[-1] += ae
    o_p, e_p = np.array(o_p), np.array(e_p)
    if len(o_p) < 2:
        return 1.0
    return stats.chisquare(o_p, e_p * o_p.sum() / e_p.sum()).pvalue


# ---------------------------------------------------------------------------
# The lattice chain written out as a finite Markov chain, from the rules:
# per-site Frank weights c_j h_j, hops at weight c_hop per molecule and
# direction into a site below capacity, everything over the total C.
# ---------------------------------------------------------------------------

def neighbours(lx, ly, s):
    x, y = s % lx, s // lx
    return [y * lx + (x + 1) % lx, y * lx + (x - 1) % lx,
            ((y + 1) % ly) * lx + x, ((y - 1) % ly) * lx + x]


def site_transitions(q, site):
    """(weight, new site counts) of the five Frank reactions in (L, D, A)."""
    L, D, A = site
    c = q["c"]
    out = [(c[0] * A, (L + 1, D, A - 1)), (c[1] * A, (L, D + 1, A - 1)),
           (c[2] * A * L, (L + 1, D, A - 1)), (c[3] * A * D, (L, D + 1, A - 1)),
           (c[4] * L * D, (L - 1, D - 1, A + 2))]
    return [(w, s) for w, s in out if w > 0]


def lattice_chain(net, q, n_mol):
    """Every lattice state with n_mol molecules and site totals <= T, and the
    sparse per-event transition weights (out of C)."""
    lx, ly, T = net["lx"], net["ly"], q["T"]
    S = lx * ly
    site_states = [(l, d, a) for l in range(T + 1) for d in range(T + 1 - l)
                   for a in range(T + 1 - l - d)]
    states = [st for st in itertools.product(site_states, repeat=S)
              if sum(map(sum, st)) == n_mol]
    index = {st: i for i, st in enumerate(states)}
    trans = []
    for i, st in enumerate(states):
        for s in range(S):
            for w, new in site_transitions(q, st[s]):
                t = list(st)
                t[s] = new
                trans.append((i, index[tuple(t)], w))
            for s2 in neighbours(lx, ly, s):
                if s2 == s or sum(st[s2]) >= T:
                    continue
                for x in range(3):
                    if st[s][x] == 0:
                        continue
                    t = [list(v) for v in st]
                    t[s][x] -= 1
                    t[s2][x] += 1
                    trans.append((i, index[tuple(map(tuple, t))], q["c_hop"] * st[s][x]))
    return states, index, trans


def exact_after_k(states, index, trans, C, start, K):
    p = [Fraction(0)] * len(states)
    p[index[start]] = Fraction(1)
    out_w = [0] * len(states)
    for i, _, w in trans:
        out_w[i] += w
    for _ in range(K):
        new = [pi * (C - ow) / C for pi, ow in zip(p, out_w)]
        for i, j, w in trans:
            if p[i]:
                new[j] += p[i] * w / C
        p = new
    return np.array([float(v) for v in p])


def empirical(orc, states, index):
    counts = np.zeros(len(states))
    for rep in orc.sites:
        counts[index[tuple(tuple(int(v) for v in site) for site in rep)]] += 1
    return counts


@pytest.mark.parametrize("lx,ly,start,K", [
    (2, 1, ((0, 0, 3), (0, 0, 1)), 5),      # x hops only; blocking at T = 3
    (1, 2, ((1, 0, 2), (0, 1, 1)), 4),      # the same along y
    (3, 1, ((0, 0, 3), (0, 0, 0), (0, 0, 0)), 4),
])
def test_fixed_k_law_of_small_lattices(lx, ly, start, K):
    net = frank_network(4, k0=0.25, k1=1.0, k2=1.0, lx=lx, ly=ly, hop=0.5, site_planes=2)
    q = quantize_lattice(net)
    assert (q["c"], q["c_hop"], q["T"]) == ([1, 1, 4, 4, 4], 2, 3)
    n_mol = sum(map(sum, start))
    states, index, trans = lattice_chain(net, q, n_mol)
    p = exact_after_k(states, index, trans, q["C"] // (lx * ly) * (lx * ly), start, K)
    n = 3000
    orc = OracleLattice(net, n * G, seed=11, stride=G)
    orc.init(("sites", np.array(start)))
    orc.step(K)
    obs = empirical(orc, states, index)
    assert chi2_p(obs, p * n) > 1e-3


def test_single_site_is_the_well_mixed_reactor():
    """On a 1x1 lattice every hop returns to its own site, so the site runs
    the well-mixed Frank chain with per-event probabilities w_j / C."""
    net = frank_network(6, k0=0.25, k1=1.0, k2=1.0, lx=1, ly=1, hop=0.5, site_planes=3)
    q = quantize_lattice(net)
    states, index, trans = lattice_chain(net, q, 6)
    start = ((0, 0, 6),)
    p = exact_after_k(states, index, trans, q["C"], start, 12)
    n = 3000
    orc = OracleLattice(net, n * G, seed=5, stride=G)
    orc.init(("sites", np.array(start)))
    orc.step(12)
    assert chi2_p(empirical(orc, states, index), p * n) > 1e-3
    assert int(orc.blocked.sum()) == 0 or q["T"] <= 6


def torus_walk(lx, ly, mu, kmax):
    """Position law of a walker stepping +-x, +-y w.p. 1/4 each after a
    Poisson(mu) number of steps, from site 0."""
    step = np.zeros((ly, lx))
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        step[dy % ly, dx % lx] += 0.25
    f = np.fft.fft2(step)
    k = np.arange(kmax)
    w = stats.poisson.pmf(k, mu)
    gen = sum(wk * f ** kk for kk, wk in zip(k, w))
    p = np.real(np.fft.ifft2(gen))
    return np.clip(p, 0, None).reshape(-1)


def test_lone_molecule_random_walk_in_time():
    """Pure diffusion: one A molecule hops to each neighbour at rate d_q, so
    after time t its site is a torus walk with Poisson(4 d_q t) steps."""
    lx, ly, t = 5, 3, 2.0
    net = frank_network(1, k0=0.0, k1=0.0, k2=0.0, lx=lx, ly=ly, hop=0.1, site_planes=4)
    q = quantize_lattice(net)
    d_q = q["c_hop"] / q["s"]
    start = np.zeros((lx * ly, 3), np.int32)
    start[0, 2] = 1
    n = 3000
    orc = OracleLattice(net, n * G, seed=3, stride=G)
    orc.init(("sites", start))
    orc.advance(t)
    pos = np.argmax(orc.sites[:, :, 2], axis=1)
    assert (orc.sites.sum(axis=(1, 2)) == 1).all()
    p = torus_walk(lx, ly, 4 * d_q * t, 80)
    obs = np.bincount(pos, minlength=lx * ly)
    assert chi2_p(obs, p * n) > 1e-3


def test_pure_diffusion_conserves_every_species():
    net = frank_network(12, k0=0.0, k1=0.0, k2=0.0, lx=6, ly=5, hop=0.1, site_planes=4)
    orc = OracleLattice(net, 64, seed=2)
    rng = np.random.default_rng(0)
    sites = np.zeros((30, 3), np.int32)
    sites[:, 0] = rng.integers(0, 5, 30)
    sites[:, 1] = rng.integers(0, 5, 30)
    sites[:, 2] = rng.integers(0, 5, 30)
    orc.init(("sites", sites))
    before = orc.totals().copy()
    orc.advance(3.0)
    assert (orc.totals() == before).all()
    assert orc.real.sum() > 0


def test_config_parameters_and_invariants():
    net = frank_network(12, lx=8, ly=8, hop=0.1, site_planes=4)
    q = quantize_lattice(net)
    assert q["c"] == [246, 246, 2048, 2048, 2048] and q["c_hop"] == 2458
    assert q["B_r"] == 18 and q["f"] == 11 and q["T"] == 15
    assert q["C"] == 64 * ((1 << 18) + 4 * 16 * 2458)
    orc = OracleLattice(net, 96, seed=1)
    orc.init(("uniform_site", 9, 15))
    n0 = orc.sites.sum(axis=(1, 2))
    orc.advance(0.5)
    assert (orc.sites.sum(axis=(1, 2)) == n0).all()
    assert (orc.sites.sum(axis=2) <= 15).all() and (orc.sites >= 0).all()
    assert orc.blocked.sum() > 0
    assert (orc.real <= orc.E).all()


def test_uniform_site_init_law():
    net = frank_network(12, lx=16, ly=16, hop=0.1, site_planes=4)
    orc = OracleLattice(net, 200, seed=9)
    orc.init(("uniform_site", 9, 15))
    a = orc.sites[:, :, 2].reshape(-1)
    assert (orc.sites[:, :, :2] == 0).all()
    obs = np.bincount(a - 9, minlength=7)
    assert len(obs) == 7
    assert chi2_p(obs, np.full(7, len(a) / 7)) > 1e-3
    # neighbouring sites and replicas are independent
    pair = (orc.sites[:, :-1, 2] - 9) * 7 + (orc.sites[:, 1:, 2] - 9)
    assert chi2_p(np.bincount(pair.reshape(-1), minlength=49),
                  np.full(49, pair.size / 49)) > 1e-3


def test_component_draw_is_uniform():
    C = 7
    ks = np.array([lattice.component(0, 0, 0, e, C) for e in range(21000)])
    assert ks.max() < C
    assert chi2_p(np.bincount(ks, minlength=C), np.full(C, len(ks) / C)) > 1e-3
    C = 1718091776
    ks = np.array([lattice.component(0, 0, 1, e, C) for e in range(20000)])
    assert ks.max() < C
    obs = np.bincount((ks * 16) // C, minlength=16)
    assert chi2_p(obs, np.full(16, len(ks) / 16)) > 1e-3


def test_group_shares_components_and_groups_differ():
    C = 1000003
    a = [lattice.component(7, 3, 0, e, C) for e in range(64)]
    b = [lattice.component(7, 3, 1, e, C) for e in range(64)]
    assert a != b
    net = frank_network(12, lx=4, ly=4, hop=0.1, site_planes=4)
    whole = OracleLattice(net, 2 * G + 5, seed=4, first=G - 3, count=8)
    whole.init(("uniform_site", 9, 15))
    whole.step(300)
    # replicas run one at a time give the same sites
    for k in range(8):
        one = OracleLattice(net, 2 * G + 5, seed=4, first=G - 3 + k, count=1)
        one.init(("uniform_site", 9, 15))
        one.step(300)
        assert (one.sites[0] == whole.sites[k]).all()
