"""Pins for the oracle's GI -> QUBO -> Ising mapping (CPU only)."""

import itertools

import numpy as np
import pytest

from oracle import gi, ssqa
from synth import random_gi_pair, random_graph


def all_assignments(N):
    idx = np.arange(2 ** N, dtype=np.int64)
    return ((idx[:, None] >> np.arange(N)) & 1).astype(np.int64)


@pytest.mark.parametrize("n,seed", [(3, 0), (3, 4), (4, 1), (4, 2)])
def test_qubo_matches_eq8_term_by_term(n, seed):
    """Eq. 8 evaluated literally equals x^T Q x + 2 n C1, for every x (n <= 3) or a
    random sample of x (n = 4)."""
    pair = random_gi_pair(n, 0.5, seed)
    for c1, c2 in [(1, 1), (2, 3)]:
        Q, const = gi.qubo_gi(pair.a1, pair.a2, c1, c2)
        assert np.array_equal(Q, np.triu(Q))
        xs = all_assignments(n * n)
        if n == 4:
            xs = xs[np.random.default_rng(seed).choice(len(xs), 400, replace=False)]
        for x in xs:
            assert gi.eq8_direct(pair.a1, pair.a2, x, c1, c2) == gi.qubo_value(Q, x) + const


@pytest.mark.parametrize("scale", [4, 12])
def test_ising_energy_is_scaled_qubo_minus_constant(scale):
    """sigma = 2x - 1 and the mapping of Section 4.2: S * H_QUBO(x) = E~(sigma) + S c."""
    pair = random_gi_pair(4, 0.5, 3)
    Q, const = gi.qubo_gi(pair.a1, pair.a2)
    h, J, c_scaled = gi.ising_from_qubo(Q, scale)
    assert np.array_equal(J, J.T) and not np.diag(J).any()
    xs = all_assignments(16)[::97]
    for x in xs:
        sigma = 2 * x - 1
        assert scale * gi.qubo_value(Q, x) == gi_energy(h, J, sigma) + c_scaled


def gi_energy(h, J, sigma):
    return ssqa.energy_direct(h, J, sigma)


@pytest.mark.parametrize("n,seed", [(3, 5), (4, 6), (4, 8)])
def test_brute_force_ground_state_and_degeneracy(n, seed):
    """Exhaustive search over all 2^N spin states: the minimum is E* and the number
    of minimisers is the number of automorphisms of graph 1 (every isomorphism is
    one ground state)."""
    pair = random_gi_pair(n, 0.5, seed)
    h, J, e_star = gi.gi_ising(pair.a1, pair.a2, 12)
    sig = 2 * all_assignments(n * n) - 1
    e = -(sig @ h) - 0.5 * np.einsum("si,ij,sj->s", sig, J.astype(np.float64), sig)
    e = np.rint(e).astype(np.int64)
    assert e.min() == e_star
    n_min = int((e == e_star).sum())
    assert n_min == gi.automorphism_count(pair.a1)
    nx = pytest.importorskip("networkx")
    g1 = nx.from_numpy_array(pair.a1)
    assert n_min == sum(1 for _ in nx.algorithms.isomorphism.GraphMatcher(g1, g1).isomorphisms_iter())


@pytest.mark.parametrize("n,seed", [(5, 0), (10, 11), (20, 1), (50, 2)])
def test_closed_form_ground_energy(n, seed):
    """Closed-form E* (from counting Q's entries) equals the energy of the known
    isomorphism x[u, perm[u]] = 1 and gi_ising's E*."""
    pair = random_gi_pair(n, 0.5, seed)
    m = pair.edges
    e_cf = gi.ground_energy_closed_form(n, m, 12)
    if n <= 20:
        h, J, e_star = gi.gi_ising(pair.a1, pair.a2, 12)
        assert e_star == e_cf
        sigma = 2 * gi.assignment_from_perm(pair.perm) - 1
        F = ssqa.field(J, sigma[None])
        assert int(ssqa.energy_from_field(h, sigma[None], F)[0]) == e_cf
    if n == 50:
        h, J, e_star = gi.gi_ising(pair.a1, pair.a2, 12)
        sigma = 2 * gi.assignment_from_perm(pair.perm) - 1
        F = ssqa.field(J, sigma[None])
        assert e_star == e_cf == int(ssqa.energy_from_field(h, sigma[None], F)[0])


def test_isomorphic_pair_and_edge_count():
    """G2 is a relabelled copy; G(5, 0.5) has five edges on average (Section 4.2)."""
    nx = pytest.importorskip("networkx")
    pair = random_gi_pair(12, 0.5, 9)
    assert nx.is_isomorphic(nx.from_numpy_array(pair.a1), nx.from_numpy_array(pair.a2))
    rng = np.random.default_rng(0)
    counts = [int(np.triu(random_graph(5, 0.5, rng), 1).sum()) for _ in range(4000)]
    assert abs(np.mean(counts) - 5.0) < 0.1


def test_coefficient_ranges_at_scale_12():
    """At S = 12 with C1 = C2 = 1 every coupling is 0, -3 or -6 (fits one int8 plane)."""
    pair = random_gi_pair(8, 0.5, 4)
    h, J, _ = gi.gi_ising(pair.a1, pair.a2, 12)
    assert set(np.unique(J).tolist()) <= {0, -3, -6}
    assert h.dtype == np.int64
