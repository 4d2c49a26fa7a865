"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random graphs, permutations, random integer Ising
coefficients and arrival times.  It holds none of the annealing arithmetic
(no QUBO, no Ising mapping, no schedules, no update rule): the oracle and the
HIP library each implement those on their own.
"""

from .graphs import (
    GIPair,
    random_graph,
    random_gi_pair,
    uneven_gi_batch,
    random_ising,
    poisson_arrivals,
)
from .workloads import WORKLOADS, Workload

__all__ = [
    "GIPair",
    "random_graph",
    "random_gi_pair",
    "uneven_gi_batch",
    "random_ising",
    "poisson_arrivals",
    "WORKLOADS",
    "Workload",
]
