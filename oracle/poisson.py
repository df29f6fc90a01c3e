"""Event budgets of the uniformised chain — oracle version.

Test infrastructure only (see the package docstring).

Because the ghost reactions make the total propensity a state-independent
constant (Eq. (9)), the waiting times of Eq. (8) form a Poisson process that
does not depend on which reactions fire.  With the padded total W = 2^B the
number of events in a time interval dt is Poisson with mean
mu = Lambda * dt, Lambda = W / s, independent of the jump chain.  Each
replica therefore draws its number of events for an advance from one 64-bit
uniform u by inversion:

    T[j] = floor(2^64 * P(K <= k_lo + j)),  j = 0 .. L-1,
    K    = k_lo + #{ j : T[j] <= u }.

k_lo is the smallest k with T >= 1 and k_lo + L - 1 the smallest k with
T = 2^64 - 1.  Here the CDF is evaluated with mpmath at 256-bit precision.
"""

import bisect

import mpmath

_PREC = 256
_TWO64 = 1 << 64


def poisson_table(mu):
    """Return (k_lo, T) for mean mu (a binary64 value taken as exact)."""
    mu = float(mu)
    if mu < 0 or mu != mu:
        raise ValueError("negative mean")
    if mu == 0.0:
        return 0, [_TWO64 - 1]
    with mpmath.workprec(_PREC):
        m = mpmath.mpf(mu)
        mode = int(mu)
        logp = -m + mode * mpmath.log(m) - mpmath.loggamma(mode + 1)
        p_mode = mpmath.exp(logp)
        tiny = mpmath.mpf(2) ** -200
        # pmf below the mode, down to where the remaining tail is negligible
        lower = []
        p = p_mode
        k = mode
        while k > 0:
            p = p * k / m          # p(k-1) = p(k) * k / mu
            k -= 1
            lower.append(p)
            if p < tiny and k < m:
                break
        lower.reverse()
        k_start = mode - len(lower)
        # pmf from the mode upward
        upper = [p_mode]
        p = p_mode
        k = mode
        while True:
            k += 1
            p = p * m / k          # p(k) = p(k-1) * mu / k
            upper.append(p)
            if p < tiny and k > m:
                break
        pmf = lower + upper
        scale = mpmath.mpf(_TWO64)
        F = mpmath.mpf(0)
        T = []
        k_lo = None
        for j, pj in enumerate(pmf):
            F += pj
            t = int(mpmath.floor(F * scale))
            if t >= _TWO64:
                t = _TWO64 - 1
            k = k_start + j
            if k_lo is None:
                if t >= 1:
                    k_lo = k
                else:
                    continue
            T.append(t)
            if t == _TWO64 - 1:
                break
        else:
            raise RuntimeError("table did not reach 2^64 - 1")
    return k_lo, T


def draw_budget(table, u):
    """K for one 64-bit uniform u."""
    k_lo, T = table
    return k_lo + bisect.bisect_right(T, u)
