"""Seeded random 3-species networks of order 1 or 2 (molecule count
conserved): the inputs of the general bit-sliced kernel's tests.

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


__all__ = ["random_network", "SPECIES"]
