"""Deterministic rate-equation limit — TEST INFRASTRUCTURE ONLY.

For large N_tot the replica mean of the counts follows the mass-action rate
equations d<N>/dt = sum_j nu_j (w_j(<N>) / s), with w_j = c_j h_j the integer
weights of quantize.py and the pair factor N(N-1)/2 taken at the mean.  The
paper's introduction contrasts this continuous description with the discrete
stochastic one the Gillespie method samples (Sec. 1).
"""

import numpy as np
from scipy.integrate import solve_ivp

from .quantize import state_change


def _h(rv, x):
    v = 1.0
    for r, n in zip(rv, x):
        if r == 1:
            v *= n
        elif r == 2:
            v *= n * (n - 1.0) / 2.0
    return v


def mean_trajectory(net, q, x0, t_eval):
    nu = np.array(state_change(net), dtype=np.float64)
    rates = np.array(q["c"], dtype=np.float64) / q["s"]

    def rhs(_t, x):
        a = np.array([k * _h(rv, x) for k, rv in zip(rates, net["reactants"])])
        return nu.T @ a

    sol = solve_ivp(rhs, (0.0, float(t_eval[-1])), np.asarray(x0, float),
                    t_eval=t_eval, rtol=1e-10, atol=1e-8, method="LSODA")
    return sol.y.T
