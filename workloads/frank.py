"""Frank-model workloads: network tables, sizes and seeded draws.

Species order everywhere is (L, D, A): the two enantiomers and the achiral
activator of Sec. 2 of the paper (the paper writes R for the second
enantiomer; it is D here).

A network is a plain dict:
  species   : tuple of names
  reactants : list of per-reaction tuples of reactant multiplicities
  products  : list of per-reaction tuples of product multiplicities
  rates     : list of mass-action rate constants (float)
  n_tot     : conserved molecule count per replica (nominal per site on a lattice)
  lx, ly    : 0, 0 for a well-mixed reactor, else a periodic lattice
  hop_rates : per-species hop rate per molecule and per direction (lattice)
  site_planes : bits per species count on a lattice site
  exact_integer : rates are already the integer weights (paper mode)
"""

import math

import numpy as np

SPECIES = ("L", "D", "A")

# Reaction vectors over (L, D, A).
_A_TO_L = ((0, 0, 1), (1, 0, 0))
_A_TO_D = ((0, 0, 1), (0, 1, 0))
_AL_TO_2L = ((1, 0, 1), (2, 0, 0))
_AD_TO_2D = ((0, 1, 1), (0, 2, 0))
_LD_TO_2A = ((1, 1, 0), (0, 0, 2))
_LL_GHOST = ((2, 0, 0), (2, 0, 0))
_DD_GHOST = ((0, 2, 0), (0, 2, 0))
_AA_GHOST = ((0, 0, 2), (0, 0, 2))


def _net(reactions, rates, n_tot, **kw):
    net = {
        "species": SPECIES,
        "reactants": [r[0] for r in reactions],
        "products": [r[1] for r in reactions],
        "rates": [float(k) for k in rates],
        "n_tot": int(n_tot),
        "lx": 0,
        "ly": 0,
        "hop_rates": [0.0, 0.0, 0.0],
        "site_planes": 0,
        "exact_integer": False,
    }
    net.update(kw)
    return net


def frank_network(n_tot, k0=0.01, k1=None, k2=None, lx=0, ly=0, hop=0.0,
                  site_planes=0):
    """Frank model with spontaneous conversion: A->L, A->D (k0), A+L->2L,
    A+D->2D (k1), L+D->2A (k2), in this table order.  k1 and k2 default to
    1/n_tot."""
    k1 = 1.0 / n_tot if k1 is None else k1
    k2 = 1.0 / n_tot if k2 is None else k2
    return _net([_A_TO_L, _A_TO_D, _AL_TO_2L, _AD_TO_2D, _LD_TO_2A],
                [k0, k0, k1, k1, k2], n_tot, lx=lx, ly=ly,
                hop_rates=[hop, hop, hop], site_planes=site_planes)


def paper_network(n_tot, ghosts=True):
    """The paper's network (Sec. 2, Eqs. (1)-(6)): autocatalysis and
    inhibition with k_A = k_I = 1, followed by the three ghost reactions that
    make the total propensity N_tot(N_tot-1)/2.  Rates are integer weights."""
    reactions = [_AL_TO_2L, _AD_TO_2D, _LD_TO_2A]
    rates = [1, 1, 1]
    if ghosts:
        reactions += [_LL_GHOST, _DD_GHOST, _AA_GHOST]
        rates += [1, 1, 1]
    return _net(reactions, rates, n_tot, exact_integer=True)


# ---------------------------------------------------------------------------
# Named workloads.  "init" is ("fixed", (L, D, A)), ("multinomial",) or
# ("uniform_site", lo, hi).
# ---------------------------------------------------------------------------

CONFIGS = {
    # Well-mixed, N_tot = 32, 1024 replicas, all-A start, t_end = 50.
    "c0": dict(net=lambda: frank_network(32), replicas=1024, seed=0, net_id=0,
               init=("fixed", (0, 0, 32)), t_end=50.0),
    # Paper-exact network, N_tot = 32, multinomial racemic start, fixed K.
    "c0p": dict(net=lambda: paper_network(32), replicas=64, seed=0, net_id=0,
                init=("multinomial",), steps=100000),
    # Well-mixed, N_tot = 1024, 2^20 replicas, all-A start, t_end = 100.
    "c1": dict(net=lambda: frank_network(1024), replicas=1 << 20, seed=0,
               net_id=0, init=("fixed", (0, 0, 1024)), t_end=100.0),
    # 64x64 periodic lattice, 12 molecules per site on average (4 planes per
    # species per site), hops at d = 0.1, 2^16 replicas, t_end = 20.
    "c2": dict(net=lambda: frank_network(12, lx=64, ly=64, hop=0.1,
                                         site_planes=4),
               replicas=1 << 16, seed=0, net_id=0,
               init=("uniform_site", 9, 15), t_end=20.0),
}


def config(name):
    c = dict(CONFIGS[name])
    c["net"] = c["net"]()
    return c


def batch_networks(n_networks=256, seed=3):
    """Uneven batch: N_tot log-uniform in [16, 4096], replicas log-uniform in
    [2^10, 2^18], k0 uniform in [1e-3, 1e-1], k1 = k2 = 1/N_tot, t_end uniform
    in [10, 200], all-A start; network i has net_id i and seed 0."""
    rng = np.random.default_rng(seed)
    n_tot = np.rint(np.exp(rng.uniform(math.log(16), math.log(4096), n_networks)))
    reps = np.rint(np.exp(rng.uniform(math.log(2 ** 10), math.log(2 ** 18), n_networks)))
    k0 = rng.uniform(1e-3, 1e-1, n_networks)
    t_end = rng.uniform(10.0, 200.0, n_networks)
    out = []
    for i in range(n_networks):
        n = int(n_tot[i])
        out.append(dict(net=frank_network(n, k0=float(k0[i])),
                        replicas=int(reps[i]), seed=0, net_id=i,
                        init=("fixed", (0, 0, n)), t_end=float(t_end[i])))
    return out


def serve_requests(rate=200.0, duration=60.0, lattice_frac=0.3, seed=4,
                   max_requests=None):
    """Served stream: Poisson arrivals; each request is a well-mixed network
    drawn as in the uneven batch, or (with probability lattice_frac) a lattice
    of side L uniform in {16..64} with the 64x64 lattice's per-site
    parameters and t_end = 20."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        if max_requests is not None and len(reqs) >= max_requests:
            break
        reps = int(np.rint(np.exp(rng.uniform(math.log(2 ** 10), math.log(2 ** 18)))))
        if rng.uniform() < lattice_frac:
            side = int(rng.integers(16, 65))
            net = frank_network(12, lx=side, ly=side, hop=0.1, site_planes=4)
            init = ("uniform_site", 9, 15)
            t_end = 20.0
            reps = max(32, reps >> 6)
        else:
            n = int(np.rint(np.exp(rng.uniform(math.log(16), math.log(4096)))))
            net = frank_network(n, k0=float(rng.uniform(1e-3, 1e-1)))
            init = ("fixed", (0, 0, n))
            t_end = float(rng.uniform(10.0, 200.0))
        reqs.append(dict(arrival=t, net=net, replicas=reps, seed=0,
                         net_id=len(reqs), init=init, t_end=t_end))
    return reqs
