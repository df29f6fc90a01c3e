"""Exact master-equation distributions for small N_tot — TEST INFRASTRUCTURE.

The Gillespie method samples the chemical master equation (Sec. 1, Sec. 3).
For small N_tot the whole state space {N : sum N = N_tot} is enumerated and
the distribution is computed directly from the reaction table, with no
sampling:

  * per event of the uniformised chain (fixed-K mode): reaction j fires with
    probability w_j(N)/W, otherwise nothing happens, so
    p_{k+1} = p_k (W I + Q_w) / W with Q_w the integer weight generator.
    Numerators are kept as Python integers over the common denominator W^k,
    so p_K is exact (dyadic rationals).
  * at time t (advance mode): the number of events is Poisson(Lambda t)
    independent of the jump chain, so p(t) = sum_k Pois(k; Lambda t) p_k.
    This is the continuous-time master equation with rates w_j / s.
"""

import math

import numpy as np

from .quantize import combinatorial_factor, state_change


def _compositions(n, S):
    if S == 1:
        return [(n,)]
    return [(a,) + rest for a in range(n + 1) for rest in _compositions(n - a, S - 1)]


def states(n_tot, n_species=3, open_net=False):
    """The state space: the simplex sum N = n_tot (closed networks; for 3
    species in the order (a, b, n_tot - a - b)), or the box [0, n_tot]^S of an
    open network."""
    if open_net:
        return [tuple(int(v) for v in s)
                for s in np.ndindex(*([n_tot + 1] * n_species))]
    if n_species == 3:
        return [(a, b, n_tot - a - b) for a in range(n_tot + 1)
                for b in range(n_tot - a + 1)]
    return _compositions(n_tot, n_species)


def weight_generator(net, q):
    """Sparse integer generator: list of (from, to, weight).  In an open
    network a firing that would pass the cap n_tot is no transition."""
    open_net = bool(net.get("open"))
    st = states(net["n_tot"], len(net["species"]), open_net)
    index = {s: i for i, s in enumerate(st)}
    nu = state_change(net)
    trans = []
    for i, s in enumerate(st):
        for j, rv in enumerate(net["reactants"]):
            w = q["c"][j] * combinatorial_factor(rv, s)
            if w == 0 or not any(nu[j]):
                continue
            t = tuple(a + d for a, d in zip(s, nu[j]))
            if open_net and max(t) > net["n_tot"]:
                continue
            trans.append((i, index[t], w))
    return st, index, trans


def fixed_k_exact(net, q, p0_state, K):
    """Exact distribution after K uniformised events from one state.
    Returns (states, numerators, denominator) with p = num / den."""
    st, index, trans = weight_generator(net, q)
    W = q["W"]
    num = [0] * len(st)
    num[index[tuple(p0_state)]] = 1
    out_w = [0] * len(st)
    for i, _, w in trans:
        out_w[i] += w
    for _ in range(K):
        new = [n * (W - ow) for n, ow in zip(num, out_w)]
        for i, t, w in trans:
            if num[i]:
                new[t] += num[i] * w
        num = new
    return st, num, W ** K


def fixed_k_probs(net, q, p0_state, K):
    st, num, den = fixed_k_exact(net, q, p0_state, K)
    # exact rational -> float via integer division at 60 extra bits
    probs = np.array([float((n << 60) // den) / float(1 << 60) for n in num])
    return st, probs


def time_probs(net, q, p0, t):
    """Distribution at time t from an initial distribution p0 (dict state ->
    probability), in binary64."""
    st, index, trans = weight_generator(net, q)
    W = float(q["W"])
    mu = q["Lambda"] * t
    p = np.zeros(len(st))
    for s, v in p0.items():
        p[index[tuple(s)]] += v
    out_w = np.zeros(len(st))
    for i, _, w in trans:
        out_w[i] += w
    src = np.array([i for i, _, _ in trans], dtype=np.int64)
    dst = np.array([t_ for _, t_, _ in trans], dtype=np.int64)
    wv = np.array([w for _, _, w in trans], dtype=np.float64) / W
    stay = 1.0 - out_w / W
    res = np.zeros(len(st))
    k = 0
    logpk = -mu
    acc = 0.0
    kmax = int(mu + 40.0 * math.sqrt(mu + 1.0) + 50)
    while k <= kmax:
        pk = math.exp(logpk)
        res += pk * p
        acc += pk
        nxt = p * stay
        np.add.at(nxt, dst, p[src] * wv)
        p = nxt
        k += 1
        logpk += math.log(mu) - math.log(k)
    return st, res


def multinomial_probs(n_tot, probs):
    """Multinomial law over (L, D, A) states."""
    st = states(n_tot)
    out = []
    for s in st:
        coef = math.factorial(n_tot)
        v = 1.0
        for k, p in zip(s, probs):
            coef //= math.factorial(k)
            v *= p ** k
        out.append(coef * v)
    return st, np.array(out)
