"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  Each checks the oracle against something
other than itself: published known-answer vectors, identities printed in the
paper, exhaustive enumeration, closed-form laws and exact master-equation
distributions.
"""

import itertools
import math

import numpy as np
import pytest
from scipy import stats

from golden import philox_kat
from oracle import master, ode, ssa
from oracle.philox import philox4x32, event_threshold
from oracle.poisson import poisson_table, draw_budget
from oracle.quantize import quantize, weights, state_change, combinatorial_factor
from workloads import frank_network, paper_network


def chi2_pvalue(observed, expected, min_expected=5.0):
    """Pearson chi-square with cells of small expectation pooled."""
    observed = np.asarray(observed, float)
    expected = np.asarray(expected, float)
    order = np.argsort(expected)
    obs_p, exp_p = [], []
    acc_o = acc_e = 0.0
    for i in order:
        acc_o += observed[i]
        acc_e += expected[i]
        if acc_e >= min_expected:
            obs_p.append(acc_o)
            exp_p.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and exp_p:
        obs_p[-1] += acc_o
        exp_p[-1] += acc_e
    obs_p, exp_p = np.array(obs_p), np.array(exp_p)
    stat = ((obs_p - exp_p) ** 2 / exp_p).sum()
    dof = max(1, len(obs_p) - 1)
    return stats.chi2.sf(stat, dof)


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

def test_philox_known_answers_python():
    for ctr, key, out in philox_kat():
        assert philox4x32(ctr, key) == out


def test_philox_known_answers_c(oracle_lib):
    for ctr, key, out in philox_kat():
        seed = key[0] | (key[1] << 32)
        assert ssa.philox_c(ctr, seed) == out


def test_event_threshold_is_uniform():
    # bits of the per-replica thresholds are fair and pairwise uncorrelated
    B = 12
    vals = np.array([event_threshold(7, 3, i, e, B)
                     for i in range(64) for e in range(64)])
    bits = (vals[:, None] >> np.arange(B)) & 1
    assert abs(bits.mean() - 0.5) < 0.02
    hist = np.bincount(vals >> 8, minlength=16)
    assert chi2_pvalue(hist, np.full(16, len(vals) / 16)) > 1e-4


# --------------------------------------------------------------------------
# Propensities, state changes and selection (Sec. 2, Sec. 3, App. A)
# --------------------------------------------------------------------------

def _simplex(n):
    for l in range(n + 1):
        for d in range(n - l + 1):
            yield (l, d, n - l - d)


def test_total_propensity_with_ghosts_is_pair_count():
    # Eq. (9): with the three ghost reactions the propensities add up to
    # N_tot (N_tot - 1) / 2 in every state.
    for n in range(0, 65):
        net = paper_network(max(n, 1))
        q = {"c": [1] * 6}
        for s in _simplex(n):
            assert sum(weights(net, q, s)) == n * (n - 1) // 2


def test_state_change_vectors_match_paper():
    # Eq. (14), species order (L, D, A)
    nu = state_change(paper_network(8))
    assert nu[:3] == [(1, 0, -1), (0, 1, -1), (-1, -1, 2)]
    assert nu[3:] == [(0, 0, 0)] * 3


def _app_a(r, a, N):
    """The serial propensity updates printed in App. A, Eqs. (A.1)-(A.3),
    for the paper's weights a = (a1..a6) and pre-reaction N = (L, D, A)."""
    L, D, A = N
    a1, a2, a3, a4, a5, a6 = a
    if r == 0:
        return (a1 - L + A - 1, a2 - D, a3 + D, a4 + L, a5, a6 - A + 1)
    if r == 1:
        return (a1 - L, a2 - D + A - 1, a3 + L, a4, a5 + D, a6 - A + 1)
    return (a1 - A + 2 * L - 2, a2 + 2 * D - A - 2, a3 - L - D + 1,
            a4 - L + 1, a5 - D + 1, a6 + 2 * A + 1)


def test_incremental_updates_of_appendix_a():
    net = paper_network(8)
    q = {"c": [1] * 6}
    nu = state_change(net)
    for n in range(1, 41):
        for s in _simplex(n):
            a = weights(net, q, s)
            for r in range(3):
                if a[r] == 0:
                    continue
                s2 = tuple(x + d for x, d in zip(s, nu[r]))
                assert tuple(weights(net, q, s2)) == _app_a(r, a, s), (n, s, r)


@pytest.mark.parametrize("netf,states", [
    (lambda: paper_network(32), [(5, 9, 18), (0, 0, 32), (16, 16, 0), (1, 30, 1)]),
    (lambda: frank_network(12), [(3, 4, 5), (0, 0, 12), (6, 0, 6)]),
])
def test_selection_by_exhaustive_thresholds(oracle_lib, netf, states):
    # The CDF search picks reaction r for exactly w_r of the W thresholds and
    # the null event for the rest (Eqs. (10)-(11), with the padded total).
    net = netf()
    q = quantize(net)
    W = q["W"]
    for s in states:
        w = weights(net, q, s)
        cnt = {}
        prev = None
        for n in range(W):
            r = ssa.select(net, q, s, n)
            cnt[r] = cnt.get(r, 0) + 1
            # thresholds map to reactions in table order, never backwards
            if prev is not None and prev >= 0:
                assert r == -1 or r >= prev
            prev = r
        for j, wj in enumerate(w):
            assert cnt.get(j, 0) == wj
        assert cnt.get(-1, 0) == W - sum(w)


def test_quantized_weights_of_the_workloads():
    # c_u = rint(k0 s): 0.01 * 16384 = 163.84 -> 164; bimolecular weights are
    # 2^f exactly because k1 = k2 = 1/N_tot is the reference rate.
    q0 = quantize(frank_network(32))
    assert q0["c"] == [164, 164, 512, 512, 512] and q0["f"] == 9
    assert q0["s"] == 16384.0 and q0["Lambda"] == 16.0
    q1 = quantize(frank_network(1024))
    assert q1["c"] == [164, 164, 16, 16, 16] and q1["B"] == 23
    assert q1["b"] == 11 and q1["Lambda"] == 512.0
    # the largest total weight, by brute force over the simplex
    for n, q in ((32, q0), (60, quantize(frank_network(60)))):
        net = frank_network(n)
        best = max(sum(weights(net, q, s)) for s in _simplex(n))
        assert best == q["max_total"]
        assert 2 ** (q["B"] - 1) < best <= 2 ** q["B"]
    qp = quantize(paper_network(32))
    assert qp["c"] == [1] * 6 and qp["B"] == 9   # 496 <= 512


# --------------------------------------------------------------------------
# Event budgets (Poisson clock of the padded total)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mu", [1e-3, 0.5, 3.0, 800.0, 51200.0])
def test_poisson_table_against_library_cdf(mu):
    k_lo, T = poisson_table(mu)
    ks = np.arange(k_lo, k_lo + len(T))
    cdf = stats.poisson.cdf(ks, mu)
    assert np.max(np.abs(np.array(T, dtype=float) / 2.0 ** 64 - cdf)) < 1e-12
    assert all(T[i] <= T[i + 1] for i in range(len(T) - 1))
    assert T[0] >= 1 and T[-1] == 2 ** 64 - 1
    # first entry: P(K <= k_lo) = e^-mu sum_{k<=k_lo} mu^k/k! (closed form)
    if k_lo == 0:
        assert abs(T[0] / 2.0 ** 64 - math.exp(-mu)) < 1e-15


def test_poisson_budget_moments():
    mu = 37.5
    tab = poisson_table(mu)
    rng = np.random.default_rng(1)
    u = rng.integers(0, 2 ** 63, 200000, dtype=np.int64).astype(np.uint64) * 2
    K = np.array([draw_budget(tab, int(x)) for x in u])
    assert abs(K.mean() - mu) < 5 * math.sqrt(mu / len(K))
    assert abs(K.var() / mu - 1) < 0.03


# --------------------------------------------------------------------------
# Whole-chain laws
# --------------------------------------------------------------------------

def test_paper_network_is_frozen_from_all_activator(oracle_lib):
    # Every reaction needs an L or a D: from (0, 0, N) only the A + A ghost
    # fires, so the state never changes.
    net = paper_network(32)
    E = ssa.OracleEnsemble(net, 256)
    E.init(("fixed", (0, 0, 32)))
    E.step(5000)
    assert (E.counts == np.array([0, 0, 32])).all()
    assert (E.real == 0).all()


def test_c_oracle_matches_python_oracle(oracle_lib):
    for net, init in ((frank_network(12), (2, 3, 7)), (paper_network(9), (3, 3, 3))):
        q = quantize(net)
        for draw in (ssa.DRAW_EVENT, ssa.DRAW_PLAIN):
            counts = np.tile(np.array(init, np.int32), (40, 1))
            E0 = np.arange(40, dtype=np.uint64) * 3
            K = np.full(40, 60, dtype=np.uint64)
            out, real, traj = ssa.run_events(net, q, 5, 2, 30, counts, E0, K,
                                             draw=draw, traj_len=60)
            for k in range(40):
                N, picked = ssa.py_events(net, q, 5, 2, 30 + k, init, int(E0[k]),
                                          60, draw=draw)
                assert list(out[k]) == N
                nu = state_change(net)
                assert int(real[k]) == sum(1 for r in picked if r >= 0 and any(nu[r]))


def test_pure_conversion_is_multinomial(oracle_lib):
    # With k1 = k2 = 0 each A turns into L or D independently at rate k0, so
    # at time t the counts are Multinomial(N; p, p, 1 - 2p),
    # p = (1 - exp(-2 k0 t)) / 2, with k0 the quantised rate c_u / s.
    n, t = 20, 5.0
    net = frank_network(n, k0=0.05, k1=0.0, k2=0.0)
    q = quantize(net)
    k0q = q["c"][0] / q["s"]
    p = (1 - math.exp(-2 * k0q * t)) / 2
    E = ssa.OracleEnsemble(net, 8192, seed=11)
    E.init(("fixed", (0, 0, n)))
    E.advance(t)
    st, probs = master.multinomial_probs(n, (p, p, 1 - 2 * p))
    idx = {s: i for i, s in enumerate(st)}
    obs = np.zeros(len(st))
    for c in E.counts:
        obs[idx[tuple(c)]] += 1
    assert chi2_pvalue(obs, probs * len(E.counts)) > 1e-4


def _empirical(counts, st):
    idx = {s: i for i, s in enumerate(st)}
    obs = np.zeros(len(st))
    for c in counts:
        obs[idx[tuple(int(x) for x in c)]] += 1
    return obs


def test_fixed_k_matches_exact_master_equation(oracle_lib):
    net = frank_network(8, k0=0.05)
    q = quantize(net)
    E = ssa.OracleEnsemble(net, 16384, seed=3)
    E.init(("fixed", (0, 0, 8)))
    K = 300
    E.step(K)
    st, probs = master.fixed_k_probs(net, q, (0, 0, 8), K)
    assert abs(probs.sum() - 1) < 1e-12
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


def test_time_mode_matches_master_equation(oracle_lib):
    net = frank_network(10, k0=0.05)
    q = quantize(net)
    E = ssa.OracleEnsemble(net, 16384, seed=4)
    E.init(("fixed", (0, 0, 10)))
    E.advance(4.0)
    E.advance(9.0)      # two advances: budgets add up as a Poisson process
    st, probs = master.time_probs(net, q, {(0, 0, 10): 1.0}, 9.0)
    assert abs(probs.sum() - 1) < 1e-9
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


# ---- the comparator's draws (PLAIN domain: one replica per thread) ----------
# The plain engine samples the same uniformised chain with its own draws: the
# low B bits of output (e mod 4) of the call keyed by e // 4.  Its law is
# pinned here directly, not by comparison with another implementation.

def test_plain_draw_fixed_k_matches_exact_master_equation(oracle_lib):
    # two steps whose lengths are not multiples of 4, so events of one
    # Philox call straddle the steps
    net = frank_network(8, k0=0.05)
    q = quantize(net)
    E = ssa.OracleEnsemble(net, 16384, seed=3, draw=ssa.DRAW_PLAIN)
    E.init(("fixed", (0, 0, 8)))
    E.step(151)
    E.step(150)
    st, probs = master.fixed_k_probs(net, q, (0, 0, 8), 301)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


def test_plain_draw_time_mode_matches_master_equation(oracle_lib):
    net = frank_network(10, k0=0.05)
    q = quantize(net)
    E = ssa.OracleEnsemble(net, 16384, seed=4, draw=ssa.DRAW_PLAIN)
    E.init(("fixed", (0, 0, 10)))
    E.advance(4.0)
    E.advance(9.0)
    st, probs = master.time_probs(net, q, {(0, 0, 10): 1.0}, 9.0)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


def test_plain_draw_paper_network_master_equation(oracle_lib):
    # unit weights, ghosts: B = 6 at N = 10, so every bit of n matters
    n = 10
    net = paper_network(n)
    q = quantize(net)
    E = ssa.OracleEnsemble(net, 16384, seed=15, draw=ssa.DRAW_PLAIN)
    E.init(("fixed", (3, 3, 4)))
    E.step(37)
    st, probs = master.fixed_k_probs(net, q, (3, 3, 4), 37)
    assert chi2_pvalue(_empirical(E.counts, st), probs * 16384) > 1e-4


@pytest.mark.parametrize("B", [5, 12, 23, 32])
def test_plain_threshold_is_uniform_and_independent(B):
    # uniform on [0, 2^B) in its top bits (a dropped top plane fails), and
    # independent between consecutive events of one call, across calls and
    # across replicas (reusing one output word, one call or one replica's
    # stream fails)
    R, K = 64, 64
    v = np.array([[ssa._ph.plain_threshold(9, 2, i, e, B) for e in range(K)]
                  for i in range(R)], dtype=np.int64)
    assert v.max() < (1 << B)
    top = v >> (B - 3)
    assert chi2_pvalue(np.bincount(top.ravel(), minlength=8), np.full(8, R * K / 8)) > 1e-4
    for a, b in ((top[:, :-1], top[:, 1:]), (top[:, :-4], top[:, 4:]),
                 (top[:-1, :], top[1:, :])):
        joint = np.bincount((8 * a + b).ravel(), minlength=64)
        assert chi2_pvalue(joint, np.full(64, a.size / 64)) > 1e-4


def test_paper_network_master_equation_from_multinomial(oracle_lib):
    # Paper-exact network, multinomial racemic start, fixed number of events.
    n = 10
    net = paper_network(n)
    q = quantize(net)
    E = ssa.OracleEnsemble(net, 16384, seed=5)
    E.init(("multinomial",))
    st, p0 = master.multinomial_probs(n, (0.25, 0.25, 0.5))
    assert chi2_pvalue(_empirical(E.counts, st), p0 * 16384) > 1e-4
    K = 200
    E.step(K)
    pK = np.zeros(len(st))
    for s, w in zip(st, p0):
        if w > 0:
            _, pk = master.fixed_k_probs(net, q, s, K)
            pK += w * pk
    assert chi2_pvalue(_empirical(E.counts, st), pK * 16384) > 1e-4


def test_homochiral_outcomes_are_symmetric(oracle_lib):
    # Sec. 6: from a racemic start the paper network ends all-L or all-D
    # (or all-A through the last inhibition), L and D equally often.
    n = 16
    net = paper_network(n)
    E = ssa.OracleEnsemble(net, 4096, seed=6)
    E.init(("multinomial",))
    E.step(4000)
    c = E.counts
    allL = int(((c[:, 0] == n)).sum())
    allD = int(((c[:, 1] == n)).sum())
    allA = int(((c[:, 2] == n)).sum())
    assert allL + allD + allA == len(c)          # absorbed
    assert stats.binomtest(allL, allL + allD, 0.5).pvalue > 1e-4


def test_mean_follows_rate_equations(oracle_lib):
    # Large N_tot: the replica mean tracks the rate equations with the
    # quantised rates, up to O(1/N_tot) corrections.
    n = 1 << 14
    net = frank_network(n)
    q = quantize(net)
    M = 32
    E = ssa.OracleEnsemble(net, M, seed=8)
    E.init(("fixed", (0, 0, n)))
    times = [1.0, 2.0, 3.0]
    means, sds = [], []
    for t in times:
        E.advance(t)
        x = E.counts / n
        means.append(x.mean(0))
        sds.append(x.std(0))
    ref = ode.mean_trajectory(net, q, [0, 0, n], np.array(times)) / n
    for m, sd, r in zip(means, sds, ref):
        tol = 5 * np.maximum(sd, 1.0 / n) / math.sqrt(M) + 4.0 / n
        assert np.all(np.abs(m - r) < tol), (m, r, tol)


def test_multinomial_initial_state(oracle_lib):
    n = 12
    c = ssa.init_multinomial(9, 1, 0, 20000, n)
    assert (c.sum(1) == n).all()
    st, p0 = master.multinomial_probs(n, (0.25, 0.25, 0.5))
    assert chi2_pvalue(_empirical(c, st), p0 * len(c)) > 1e-4


def test_histogram_rule():
    n = 10
    counts = np.array([[10, 0, 0], [0, 10, 0], [5, 5, 0], [0, 0, 10], [6, 4, 0]])
    h = ssa.ee_histogram(counts, n, 256)
    # ee = +1 -> last bin; ee = -1 -> bin 0; ee = 0 -> bin 128; ee = 0.2 -> 153
    assert h[255] == 1 and h[0] == 1 and h[128] == 2 and h[153] == 1
    assert h.sum() == len(counts)


# ---- shared-threshold variant (one n for every copy) --------------------------

def test_shared_draw_is_uniform_on_z():
    for Z in (7, 496):
        n = np.array([ssa.draw_shared(11, 3, e, Z) for e in range(20 * Z if Z < 100 else 24800)])
        assert n.max() < Z
        bins = min(Z, 16)
        obs = np.bincount((n * bins) // Z, minlength=bins)
        exp = np.array([sum(1 for v in range(Z) if (v * bins) // Z == b) for b in range(bins)],
                       float) * len(n) / Z
        assert chi2_pvalue(obs, exp) > 1e-3


def test_shared_z_is_the_paper_total():
    """With the ghost reactions the total weight is N(N-1)/2 in every state
    (Eq. (9)); Z of the shared draw is that total, else W."""
    for n in (6, 32, 100):
        q = quantize(paper_network(n))
        assert q["z_shared"] == n * (n - 1) // 2
    q = quantize(frank_network(64))
    assert q["z_shared"] == q["W"]


def _paper_chain_law(n_tot, start, K):
    """Exact law after K events of the paper's iteration on [0, Z): reaction r
    with probability a_r / Z, a_r the propensities of Eq. (7) with k = 1
    (the ghosts keep the state)."""
    from fractions import Fraction
    Z = n_tot * (n_tot - 1) // 2
    states = [(l, d, n_tot - l - d) for l in range(n_tot + 1) for d in range(n_tot + 1 - l)]
    idx = {s: i for i, s in enumerate(states)}
    p = [Fraction(0)] * len(states)
    p[idx[start]] = Fraction(1)
    for _ in range(K):
        new = [Fraction(0)] * len(states)
        for i, (l, d, a) in enumerate(states):
            if not p[i]:
                continue
            moves = [(a * l, (l + 1, d, a - 1)), (a * d, (l, d + 1, a - 1)),
                     (l * d, (l - 1, d - 1, a + 2))]
            stay = Z - sum(w for w, _ in moves)
            new[i] += p[i] * Fraction(stay, Z)
            for w, s in moves:
                if w:
                    new[idx[s]] += p[i] * Fraction(w, Z)
        p = new
    return states, np.array([float(v) for v in p])


def test_shared_threshold_law_of_one_copy():
    """Each copy of the shared-threshold iteration is the paper's chain:
    independent seeds give independent samples of its exact law."""
    net = paper_network(6)
    q = quantize(net)
    start, K = (2, 2, 2), 12
    states, p = _paper_chain_law(6, start, K)
    idx = {s: i for i, s in enumerate(states)}
    obs = np.zeros(len(states))
    for seed in range(3000):
        o = ssa.OracleEnsemble(net, 1, seed=seed, draw=ssa.DRAW_SHARED, q=q)
        o.init(("fixed", start))
        o.step(K)
        obs[idx[tuple(int(v) for v in o.counts[0])]] += 1
    assert chi2_pvalue(obs, p * 3000) > 1e-3


def test_shared_threshold_is_one_number_per_event():
    """Every copy compares the same n at an event (C and pure Python agree),
    and copies from one state stay identical."""
    net = paper_network(32)
    q = quantize(net)
    o = ssa.OracleEnsemble(net, 40, seed=5, draw=ssa.DRAW_SHARED, q=q)
    o.init(("multinomial",))
    start = o.counts.copy()
    o.step(300)
    for k in (0, 7, 39):
        got, _ = ssa.py_events(net, q, 5, 0, k, list(start[k]), 0, 300, ssa.DRAW_SHARED)
        assert list(o.counts[k]) == got
    same = ssa.OracleEnsemble(net, 8, seed=5, draw=ssa.DRAW_SHARED, q=q)
    same.init(("fixed", (10, 10, 12)))
    same.step(500)
    assert (same.counts == same.counts[0]).all()


def _paper_chain_time_law(n_tot, start, t):
    """Law at time t of the paper's continuous-time chain (rates A L, A D,
    L D with k = 1; the ghosts change nothing): exp(Q t) applied to the
    start, Q written from the three reactions."""
    from scipy.linalg import expm
    states = [(l, d, n_tot - l - d) for l in range(n_tot + 1) for d in range(n_tot + 1 - l)]
    idx = {s: i for i, s in enumerate(states)}
    Q = np.zeros((len(states), len(states)))
    for i, (l, d, a) in enumerate(states):
        for w, s in ((a * l, (l + 1, d, a - 1)), (a * d, (l, d + 1, a - 1)),
                     (l * d, (l - 1, d - 1, a + 2))):
            if w:
                Q[idx[s], i] += w
                Q[i, i] -= w
    p0 = np.zeros(len(states))
    p0[idx[start]] = 1.0
    return states, expm(Q * t) @ p0


def test_shared_time_law_of_one_copy():
    """With one shared budget per advance (the paper's shared tau) at rate
    Z / s, each copy is the paper's continuous-time chain: 3000 independent
    seeds against exp(Q t) from (2, 2, 2) at N = 6, t = 0.25 (two advances)."""
    net = paper_network(6)
    q = quantize(net)
    start, t = (2, 2, 2), 0.25
    states, p = _paper_chain_time_law(6, start, t)
    idx = {s: i for i, s in enumerate(states)}
    obs = np.zeros(len(states))
    for seed in range(3000):
        o = ssa.OracleEnsemble(net, 1, seed=seed, draw=ssa.DRAW_SHARED, q=q)
        o.init(("fixed", start))
        o.advance(0.1)
        o.advance(t)
        obs[idx[tuple(int(v) for v in o.counts[0])]] += 1
    assert chi2_pvalue(obs, p * 3000) > 1e-3


def test_shared_budget_is_one_poisson_number_per_advance():
    """Every copy runs the same number of events in an advance, Poisson with
    mean (Z / s) (t_end - t_now): 2000 seeds against the Poisson law."""
    net = paper_network(10)
    q = quantize(net)
    rate = 45.0                               # Z = 10 * 9 / 2, s = 1
    assert q["z_shared"] / q["s"] == rate
    ks = []
    for seed in range(2000):
        o = ssa.OracleEnsemble(net, 20, seed=seed, draw=ssa.DRAW_SHARED, q=q)
        o.init(("multinomial",))
        o.advance(0.2)
        assert (o.E == o.E[0]).all()
        ks.append(int(o.E[0]))
    ks = np.array(ks)
    kmax = ks.max() + 1
    obs = np.bincount(ks, minlength=kmax + 1)
    exp = stats.poisson.pmf(np.arange(kmax + 1), rate * 0.2) * len(ks)
    exp[-1] += stats.poisson.sf(kmax, rate * 0.2) * len(ks)
    assert chi2_pvalue(obs, exp) > 1e-3


@pytest.mark.parametrize("seed,n_tot,R,integer", [(3, 6, 5, False), (5, 7, 8, False),
                                                  (11, 6, 6, True)])
def test_random_network_fixed_k_law(seed, n_tot, R, integer):
    """The oracle on seeded random 3-species networks of order <= 2 (dimers,
    pairs, no-change reactions) against the exact law after K uniformised
    events, computed from the generator's integer weights."""
    from workloads import random_network
    net = random_network(seed, n_tot, R, exact_integer=integer)
    q = quantize(net)
    start = (n_tot // 3, n_tot // 3, n_tot - 2 * (n_tot // 3))
    K = 9
    st, probs = master.fixed_k_probs(net, q, start, K)
    M = 6000
    o = ssa.OracleEnsemble(net, M, seed=seed + 100, q=q)
    o.init(("fixed", start))
    o.step(K)
    idx = {s: i for i, s in enumerate(st)}
    obs = np.zeros(len(st))
    for c in o.counts:
        obs[idx[tuple(int(v) for v in c)]] += 1
    assert chi2_pvalue(obs, probs * M) > 1e-3
