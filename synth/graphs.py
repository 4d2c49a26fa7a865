"""Random graph-isomorphism pairs and other seeded inputs.

The paper generates each GI problem by drawing a random graph in which every
vertex pair is connected with probability 0.5 and copying it into a second graph
(Section 4.2, simulation setup).  Here the copy is relabelled by a seeded random
permutation pi, A2[u, v] = A1[pi[u], pi[v]], so that the ground state is not
the trivial identity mapping; pi = identity reproduces the plain copy.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GIPair:
    """Two isomorphic graphs as 0/1 adjacency matrices.

    a1, a2: uint8 [n, n], symmetric, zero diagonal.
    perm:   int64 [n]; a2[u, v] == a1[perm[u], perm[v]], i.e. vertex u of graph 2
            corresponds to vertex perm[u] of graph 1.
    """

    a1: np.ndarray
    a2: np.ndarray
    perm: np.ndarray

    @property
    def n(self) -> int:
        return int(self.a1.shape[0])

    @property
    def edges(self) -> int:
        return int(np.triu(self.a1, 1).sum())


def random_graph(n: int, p: float, rng: np.random.Generator) -> np.ndarray:
    """G(n, p): each of the n(n-1)/2 vertex pairs is an edge with probability p."""
    upper = np.triu(rng.random((n, n)) < p, 1)
    a = (upper | upper.T).astype(np.uint8)
    return a


def random_gi_pair(n: int, p: float = 0.5, seed: int = 0) -> GIPair:
    """Seeded GI pair: G(n, p) and a randomly relabelled copy.

    The generator is ``numpy.random.default_rng(seed)``; the graph is drawn first,
    then the permutation.
    """
    rng = np.random.default_rng(seed)
    a1 = random_graph(n, p, rng)
    perm = rng.permutation(n).astype(np.int64)
    a2 = a1[np.ix_(perm, perm)].copy()
    return GIPair(a1=a1, a2=a2, perm=perm)


def uneven_gi_batch(count: int, n_lo: int = 10, n_hi: int = 50, p_lo: float = 0.3,
                    p_hi: float = 0.7, seed_base: int = 1000) -> list[GIPair]:
    """Many GI pairs of uneven size: instance g uses default_rng(seed_base + g) to
    draw n ~ U{n_lo..n_hi}, p ~ U[p_lo, p_hi], the graph and the permutation."""
    out = []
    for g in range(count):
        rng = np.random.default_rng(seed_base + g)
        n = int(rng.integers(n_lo, n_hi + 1))
        p = float(rng.uniform(p_lo, p_hi))
        a1 = random_graph(n, p, rng)
        perm = rng.permutation(n).astype(np.int64)
        a2 = a1[np.ix_(perm, perm)].copy()
        out.append(GIPair(a1=a1, a2=a2, perm=perm))
    return out


def random_ising(n: int, seed: int, h_max: int = 64, j_max: int = 7,
                 density: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Random integer Ising coefficients: h int32 [n] in [-h_max, h_max], J int32
    [n, n] symmetric with zero diagonal and entries in [-j_max, j_max] (a fraction
    ``density`` of the off-diagonal pairs non-zero)."""
    rng = np.random.default_rng(seed)
    h = rng.integers(-h_max, h_max + 1, size=n).astype(np.int32)
    vals = rng.integers(-j_max, j_max + 1, size=(n, n))
    mask = rng.random((n, n)) < density
    upper = np.triu(np.where(mask, vals, 0), 1)
    J = (upper + upper.T).astype(np.int32)
    return h, J


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times in seconds of ``count`` requests of a Poisson stream."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    return np.cumsum(gaps)
