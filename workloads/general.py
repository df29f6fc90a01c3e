"""Seeded random networks of order 1 or 2: 3-species networks that conserve
the molecule count, and networks of any species count, closed or open
(molecule count not conserved, every count capped at n_tot): the inputs of
the general bit-sliced kernels' tests and benchmark.

Each reaction takes one or two reactant molecules and gives as many product
molecules, species drawn uniformly; some reactions change nothing (like the
paper's ghost reactions).  Rates are log-uniform on [1e-3, 1].  Plain tables
only: no weights, no quantisation.
"""

import numpy as np

from .frank import SPECIES, _net


def random_network(seed, n_tot, n_reactions, exact_integer=False):
    rng = np.random.default_rng(seed)
    reactions = []
    for _ in range(n_reactions):
        order = int(rng.integers(1, 3))
        r = np.zeros(3, int)
        p = np.zeros(3, int)
        for x in rng.integers(0, 3, order):
            r[x] += 1
        if rng.random() < 0.15:
            p = r.copy()                       # changes nothing
        else:
            for x in rng.integers(0, 3, order):
                p[x] += 1
        reactions.append((tuple(int(v) for v in r), tuple(int(v) for v in p)))
    if exact_integer:
        rates = [int(k) for k in rng.integers(0, 6, n_reactions)]
        if not any(rates):
            rates[0] = 1
    else:
        rates = list(10.0 ** rng.uniform(-3, 0, n_reactions))
    return _net(reactions, rates, n_tot, exact_integer=exact_integer)


def random_wide_network(seed, n_species, n_tot, n_reactions, open_net=False):
    """A random network of n_species species (names S0, S1, ...).  Closed:
    every reaction gives as many molecules as it takes.  Open: a reaction
    gives 0 to 3 molecules (at most 2 more or fewer of any one species), so
    counts grow and shrink, capped at n_tot."""
    rng = np.random.default_rng(seed)
    S = int(n_species)
    reactions = []
    while len(reactions) < n_reactions:
        order = int(rng.integers(1, 3))
        r = np.zeros(S, int)
        for x in rng.integers(0, S, order):
            r[x] += 1
        n_out = int(rng.integers(0, 4)) if open_net else order
        p = np.zeros(S, int)
        for x in rng.integers(0, S, n_out):
            p[x] += 1
        if np.abs(p - r).max() > 2:
            continue
        reactions.append((tuple(int(v) for v in r), tuple(int(v) for v in p)))
    rates = list(10.0 ** rng.uniform(-2, 0, n_reactions))
    net = _net(reactions, rates, n_tot)
    net["species"] = tuple("S%d" % x for x in range(S))
    net["hop_rates"] = [0.0] * S
    net["open"] = bool(open_net)
    return net


def open_network(name, cap):
    """Named open networks: 'death' (A -> 0), 'birth' (A -> 2A),
    'lotka_volterra' (X -> 2X, X + Y -> 2Y, Y -> 0), counts capped at cap."""
    if name == "death":
        species, reactions, rates = ("A",), [((1,), (0,))], [0.3]
    elif name == "birth":
        species, reactions, rates = ("A",), [((1,), (2,))], [0.5]
    elif name == "lotka_volterra":
        species = ("X", "Y")
        reactions = [((1, 0), (2, 0)), ((1, 1), (0, 2)), ((0, 1), (0, 0))]
        rates = [1.0, 0.1, 0.6]
    else:
        raise ValueError(name)
    net = _net(reactions, rates, cap)
    net["species"] = species
    net["hop_rates"] = [0.0] * len(species)
    net["open"] = True
    return net


__all__ = ["random_network", "random_wide_network", "open_network", "SPECIES"]
