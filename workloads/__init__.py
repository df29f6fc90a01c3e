"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds network descriptions (stoichiometry and rate tables),
seeds, sizes and the seeded draws that define the uneven batch and the served
request stream.  It holds none of the simulation arithmetic: no quantisation,
no propensities, no random-number generator of the method.  Both the CPU
oracle and the GPU path read their inputs from here and from nowhere else.
"""

from .frank import (  # noqa: F401
    SPECIES,
    frank_network,
    paper_network,
    CONFIGS,
    config,
    batch_networks,
    serve_requests,
)
from .general import random_network, random_wide_network, open_network  # noqa: F401
