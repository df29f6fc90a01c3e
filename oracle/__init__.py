"""CPU oracle for the bit-parallel Gillespie path — TEST INFRASTRUCTURE ONLY.

Only the tests, the package entry's smoke check and the benchmark's CPU
baseline may import, call, link or execute anything in this directory.  The
product path never does: it runs the HIP library and fails loudly when that
library is missing.

What the oracle computes (each module cites the passage it follows):
  philox.py    Philox4x32-10 counter-based generator (Salmon et al., SC'11),
               pinned to the published known-answer vectors.
  quantize.py  integer reaction weights c_j, scale s, uniformisation bound
               W = 2^B and event rate Lambda from a rate table.
  poisson.py   Poisson CDF tables floor(2^64 F(k)) in 256-bit arithmetic.
  ssa.c/.py    per-replica Gillespie direct method with integer counts:
               propensities recomputed from their definition every event,
               linear CDF search, occupancy update (Sec. 3 of the paper),
               plus the pure-Python version used for tiny cases.
  master.py    exact master-equation distributions for small N_tot.
  ode.py       deterministic rate-equation limit.
  lattice.c    compartment (lattice) version of the direct method.

It shares no code with the HIP path.  The only inputs both sides read are the
seeded workloads in the top-level ``workloads`` package.
"""
