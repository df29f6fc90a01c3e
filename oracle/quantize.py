"""Integer reaction weights for an exact, bit-exact SSA — oracle version.

Test infrastructure only (see the package docstring).

The paper makes every propensity an integer by setting k_A = k_I = 1
(Sec. 2, after Eq. (6)) and leaves real-valued rates to future work
(Sec. 6).  The rule used here, for a table of mass-action rates k_j:

  * h_j(N) is the combinatorial factor of the reactants: N_X for X -> ...,
    N_X N_Y for X + Y -> ..., N_X (N_X - 1)/2 for 2X -> ... (the forms of
    Eq. (7)).
  * exact-integer tables (the paper's network) use c_j = k_j and s = 1.
  * otherwise k_ref is the largest bimolecular rate (the largest rate if
    there is no bimolecular reaction), and for f = 0, 1, 2, ... the scale is
    s = 2^f / k_ref and c_j = rint(k_j s) (IEEE binary64 product, ties to
    even); the first f at which every reaction with k_j > 0 either has an
    integral product k_j s (no rounding) or c_j >= 2^p is taken
    (p = precision_bits, default 7, so a rounded weight is off by at most
    2^-8 relative).
  * the weight of reaction j is w_j(N) = c_j h_j(N); its rate per unit time
    is w_j / s.
  * W = 2^B is the smallest power of two at or above a bound of the total
    weight sum_j w_j(N) over the state space; the uniformised chain makes
    Lambda = W / s events per unit time, each event picking reaction j with
    probability w_j / W and doing nothing otherwise.  This is the role the
    ghost reactions play in the paper: they pad the total propensity to a
    state-independent constant (Eq. (9)).  Any bound at or above the largest
    total gives the same law; the bound used is
      - 3 species, molecule count conserved (the Frank family): the largest
        total over the simplex sum_X N_X = N_tot, by enumerating it;
      - any other network: sum_j c_j max h_j, each reaction's largest factor
        over the state space: on the simplex N for N_X, floor(N/2) ceil(N/2)
        for N_X N_Y, N (N - 1) / 2 for N_X (N_X - 1) / 2; on the box of an
        open network (every count at most the cap C = N_tot) C, C^2 and
        C (C - 1) / 2 (all attained at the corner N = (C, ..., C)).
  * open networks (net["open"]: reactions need not conserve the molecule
    count, the general networks of Sec. 6): every species count is capped at
    N_tot; a selected reaction that would pass the cap does nothing (ssa.c).
"""

import math

import numpy as np


def combinatorial_factor(reactants, counts):
    """h(N) of one reaction: prod_X C(N_X, r_X) for r_X in {0, 1, 2}."""
    v = 1
    for r, n in zip(reactants, counts):
        if r == 1:
            v *= n
        elif r == 2:
            v *= n * (n - 1) // 2
        elif r != 0:
            raise ValueError("reaction order above 2")
    return v


def _validate(net):
    S = len(net["species"])
    for rv, pv in zip(net["reactants"], net["products"]):
        if len(rv) != S or len(pv) != S:
            raise ValueError("stoichiometry width")
        if sum(rv) < 1 or sum(rv) > 2:
            raise ValueError("reaction order must be 1 or 2")
        if sum(rv) != sum(pv) and not net.get("open"):
            raise ValueError("reaction does not conserve the molecule count")
        if min(rv) < 0 or min(pv) < 0:
            raise ValueError("negative stoichiometry")
    for k in net["rates"]:
        if not (k >= 0.0) or math.isinf(k):
            raise ValueError("rate must be finite and >= 0")


def _max_total_weight(net, c):
    """max over the simplex sum N = n_tot of sum_j c_j h_j(N), by enumeration
    of every state (int64; the guard keeps products far from overflow)."""
    return _total_weight_range(net, c)[1]


def _factor_max(rv, n, open_net):
    """Largest h(N) of one reaction over the simplex of n molecules, or over
    the box [0, n]^S of an open network."""
    xs = [x for x, r in enumerate(rv) for _ in range(r)]
    if len(xs) == 1:
        return n
    if xs[0] != xs[1]:
        return n * n if open_net else (n // 2) * (n - n // 2)
    return n * (n - 1) // 2


def total_weight_bound(net, c):
    """(min or None, bound): the exact (min, max) total weight over the
    simplex for 3-species closed networks, else (None, sum_j c_j max h_j)."""
    if len(net["species"]) == 3 and not net.get("open"):
        return _total_weight_range(net, c)
    n = net["n_tot"]
    return None, sum(cj * _factor_max(rv, n, net.get("open"))
                     for cj, rv in zip(c, net["reactants"]))


def _total_weight_range(net, c):
    """(min, max) over the simplex sum N = n_tot of sum_j c_j h_j(N)."""
    S = len(net["species"])
    n = net["n_tot"]
    if S != 3:
        raise ValueError("enumeration implemented for 3 species")
    if max(c + [1]) * (n + 1) * (n + 1) >= (1 << 60):
        raise ValueError("weights too large for the enumeration")
    best, least = 0, None
    for n0 in range(n + 1):
        n1 = np.arange(0, n - n0 + 1, dtype=np.int64)
        n2 = (n - n0) - n1
        cols = (np.full(n1.shape, n0, dtype=np.int64), n1, n2)
        tot = np.zeros(n1.shape, dtype=np.int64)
        for cj, rv in zip(c, net["reactants"]):
            if cj == 0:
                continue
            h = np.ones(n1.shape, dtype=np.int64)
            for r, col in zip(rv, cols):
                if r == 1:
                    h = h * col
                elif r == 2:
                    h = h * (col * (col - 1) // 2)
            tot = tot + cj * h
        best = max(best, int(tot.max()))
        least = int(tot.min()) if least is None else min(least, int(tot.min()))
    return least, best


def quantize(net, precision_bits=7, max_total=None):
    """Return dict(c, f, s, B, W, Lambda, b) for a network table."""
    _validate(net)
    rates = net["rates"]
    orders = [sum(rv) for rv in net["reactants"]]
    if net.get("exact_integer"):
        c = []
        for k in rates:
            if k != int(k):
                raise ValueError("exact-integer table with a non-integer rate")
            c.append(int(k))
        f, s = 0, 1.0
    else:
        bi = [k for k, o in zip(rates, orders) if o == 2 and k > 0]
        pos = [k for k in rates if k > 0]
        if not pos:
            raise ValueError("every rate is zero")
        k_ref = max(bi) if bi else max(pos)
        for f in range(0, 64):
            s = math.ldexp(1.0, f) / k_ref
            prod = [k * s for k in rates]
            c = [int(round(x)) for x in prod]
            if all(x == cj or cj >= (1 << precision_bits)
                   for x, cj, k in zip(prod, c, rates) if k > 0):
                break
        else:
            raise ValueError("no scale reaches the precision")
    min_total = None
    if max_total is None:
        min_total, max_total = total_weight_bound(net, c)
    B = max(1, (max_total - 1).bit_length()) if max_total > 1 else 1
    W = 1 << B
    Lam = math.ldexp(1.0, B) / s
    b = max(1, int(net["n_tot"]).bit_length())
    # Z of the shared-threshold variant: the total weight when it is the same
    # in every state (the paper's ghost reactions make it N(N-1)/2, Eq. (9)),
    # else W; None when it does not fit 32 bits
    z = max_total if (min_total is not None and min_total == max_total and max_total > 0) else W
    z_shared = z if z < (1 << 32) else None
    return dict(c=c, f=f, s=s, B=B, W=W, Lambda=Lam, b=b, max_total=max_total,
                z_shared=z_shared)


def weights(net, q, counts):
    """w_j(N) = c_j h_j(N) for every reaction, from the definition."""
    return [cj * combinatorial_factor(rv, counts)
            for cj, rv in zip(q["c"], net["reactants"])]


def state_change(net):
    """nu_j = products - reactants (Eq. (14) for the paper's reactions)."""
    return [tuple(p - r for p, r in zip(pv, rv))
            for rv, pv in zip(net["reactants"], net["products"])]
