"""The benchmark and parity workloads, as plain data.

Parameter values are the paper's SSQA defaults (Table 2: J_perp from 0 to 1/2,
beta = 3, delay d = 1, I_0 = 2, n_rnd = 1) with tau = 100 (the Fig. 5 setting).
``scale`` is the integer factor S that makes h, J, J_perp and the noise exact
integers (quarter-integer h and J from the QUBO-to-Ising mapping, sixths of
J_perp); ``alpha`` is one least-significant unit of that integer model.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # GI graph vertices; spins N = n * n
    p: float               # edge probability
    graph_seed: int
    replicas: int          # R
    trials: int            # T
    cycles: int            # SC
    seed: int              # Philox key
    tau: int = 100
    beta: int = 3
    jperp_min: Fraction = Fraction(0)
    jperp_max: Fraction = Fraction(1, 2)
    delay: int = 1
    i0: Fraction = Fraction(2)
    n_rnd: Fraction = Fraction(1)
    scale: int = 12
    alpha: int = 1
    coupling_mode: int = 0
    notes: str = field(default="")

    @property
    def spins(self) -> int:
        return self.n * self.n

    @property
    def columns(self) -> int:
        return self.replicas * self.trials

    @property
    def spin_updates(self) -> int:
        return self.spins * self.replicas * self.trials * self.cycles


WORKLOADS = {
    "gi5": Workload("gi5", n=5, p=0.5, graph_seed=0, replicas=8, trials=100, cycles=500, seed=0,
                    notes="N=25, small case"),
    "gi20": Workload("gi20", n=20, p=0.5, graph_seed=1, replicas=32, trials=256, cycles=2000, seed=0,
                     notes="N=400"),
    "gi50": Workload("gi50", n=50, p=0.5, graph_seed=2, replicas=64, trials=1024, cycles=2000, seed=0,
                     notes="N=2500, the paper's largest size"),
}
