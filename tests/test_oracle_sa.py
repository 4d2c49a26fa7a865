"""Pins of the SA baseline oracle (Section 4.4, Table 4) against things other than itself:
the library exponential, the limits of infinite and zero temperature, the Boltzmann distribution
that single-spin Metropolis samples at a fixed temperature, direct energies of Eq. 1, and the
paper's SA success at N = 25."""

import math

import numpy as np
import pytest

from oracle import gi, philox, sa
from synth import random_gi_pair, random_ising


def _direct_energy(h, J, s):
    """Eq. 1 as a double sum over i < j."""
    n = len(h)
    e = 0
    for i in range(n):
        e -= int(h[i]) * int(s[i])
        for j in range(i + 1, n):
            e -= int(J[i, j]) * int(s[i]) * int(s[j])
    return e


def test_exp_neg_matches_library_exp():
    xs = np.concatenate([np.linspace(0.0, 700.0, 30001), np.random.default_rng(0).uniform(0.0, 60.0, 30000),
                         [0.0, 1e-300, 0.5 * math.log(2), math.log(2), 700.0]])
    for x in xs:
        ref = math.exp(-x)
        assert abs(sa.exp_neg(x) - ref) <= 1e-12 * ref, x
    assert sa.exp_neg(0.0) == 1.0
    assert sa.exp_neg(700.5) == 0.0
    assert sa.accept_threshold(0, 0.3) == 2.0 ** 32
    assert sa.accept_threshold(5, 0.0) == 2.0 ** 32


def test_schedule_is_linear_in_inverse_temperature():
    """1/T(t+1) = 1/T(t) + Delta, T(0) = T_start, T(last) = T_end, at scale S."""
    b = sa.sa_schedule(40000, 1000.0, 0.1, 12)
    assert b[0] == 1.0 / 12000.0
    assert abs(b[-1] - 1.0 / 1.2) < 1e-12
    d = np.diff(b)
    assert np.allclose(d, (1.0 / 1.2 - 1.0 / 12000.0) / 39999, rtol=1e-9, atol=0)
    assert sa.sa_schedule(1, 5.0, 1.0, 4)[0] == 1.0 / 20.0


def _picks(n, cycles, b, seed):
    w0, _, _, _ = philox.philox4x32_10(np.arange(cycles), sa.SA_STEP_TAG, 0, b, seed & 0xFFFFFFFF, seed >> 32)
    return (w0 * np.uint64(n)) >> np.uint64(32)


def test_infinite_temperature_flips_every_pick():
    """beta = 0 accepts every proposal: the final state is the initial one with each spin flipped once
    per time it was picked, and every energy in the trace is Eq. 1 of the state at that time."""
    h, J = random_ising(9, 3, h_max=20, j_max=7)
    cycles, seed = 60, 11
    res = sa.sa_anneal(h, J, [0, 4], cycles, np.zeros(cycles), seed)
    for col, b in enumerate([0, 4]):
        s = sa.initial_spins(9, b, seed & 0xFFFFFFFF, seed >> 32).copy()
        assert res.trace[0, col] == _direct_energy(h, J, s)
        for t, i in enumerate(_picks(9, cycles, b, seed)):
            s[int(i)] = -s[int(i)]
            assert res.trace[t + 1, col] == _direct_energy(h, J, s)
        assert np.array_equal(res.spins[col], s)
        assert res.energy[col] == _direct_energy(h, J, s)


def test_initial_spins_follow_the_stream_layout():
    """Spin i takes bit i & 31 of word (i & 127) >> 5 of the block (i >> 7, init tag, 0, b)."""
    k0, k1 = 77, 5
    s = sa.initial_spins(300, 3, k0, k1)
    for i in (0, 1, 31, 32, 127, 128, 255, 299):
        words = philox.philox4x32_10(i >> 7, sa.SA_INIT_TAG, 0, 3, k0, k1)
        bit = (int(words[(i & 127) >> 5]) >> (i & 31)) & 1
        assert s[i] == (1 if bit else -1)


def test_zero_temperature_never_climbs():
    """beta -> infinity accepts only dE <= 0: the energy never increases, and every proposal that
    would lower the energy of the current state is taken."""
    h, J = random_ising(16, 8, h_max=30, j_max=9)
    cycles = 400
    res = sa.sa_anneal(h, J, 3, cycles, np.full(cycles, 1e300), 2)
    assert (np.diff(res.trace, axis=0) <= 0).all()
    for col in range(3):
        assert res.energy[col] == _direct_energy(h, J, res.spins[col]) == res.trace[-1, col]
        assert res.best[col] == res.trace[:, col].min()
    # the final state of a long descent is a local minimum of every spin that was proposed at the end
    s = res.spins[0].astype(np.int64)
    late = set(int(i) for i in _picks(16, cycles, 0, 2)[-100:])
    for i in late:
        de = 2 * s[i] * (h[i] + J[i] @ s)
        assert de >= 0


def test_fixed_temperature_samples_boltzmann():
    """Single-spin Metropolis with uniform proposals satisfies detailed balance: at a fixed beta the
    long-run frequency of each energy level approaches g(E) exp(-beta E) / Z (N = 3, all 8 states)."""
    h = np.array([3, -2, 1])
    J = np.array([[0, 4, -1], [4, 0, 2], [-1, 2, 0]])
    beta = 0.35
    cycles = 200000
    res = sa.sa_anneal(h, J, 1, cycles, np.full(cycles, beta), 9)
    levels = {}
    for bits in range(8):
        s = np.array([1 if bits >> k & 1 else -1 for k in range(3)])
        e = _direct_energy(h, J, s)
        levels[e] = levels.get(e, 0) + 1
    z = sum(g * math.exp(-beta * e) for e, g in levels.items())
    tr = res.trace[1000:, 0]
    for e, g in levels.items():
        assert abs((tr == e).mean() - g * math.exp(-beta * e) / z) < 0.01, e


def test_first_hit_and_best_are_consistent():
    pair = random_gi_pair(3, 0.5, 4)
    h, J, e_star = gi.gi_ising(pair.a1, pair.a2, 12)
    cycles = 3000
    beta = sa.sa_schedule(cycles, 1000.0, 0.1, 12)
    res = sa.sa_anneal(h, J, 6, cycles, beta, 1, target=e_star)
    for col in range(6):
        assert res.best[col] == res.trace[:, col].min() >= e_star
        if res.first_hit[col] >= 0:
            assert res.trace[res.first_hit[col], col] == e_star
            assert (res.trace[: res.first_hit[col], col] != e_star).all()
        else:
            assert (res.trace[:, col] != e_star).all()


@pytest.mark.timeout(300)
def test_gi_n5_success_like_table4():
    """Table 4: SA with 40,000 cycles solves N = 25 in 100 % of trials."""
    pair = random_gi_pair(5, 0.5, 0)
    h, J, e_star = gi.gi_ising(pair.a1, pair.a2, 12)
    cycles = 40000
    res = sa.sa_anneal(h, J, 8, cycles, sa.sa_schedule(cycles, 1000.0, 0.1, 12), 0, target=e_star)
    assert (res.best == e_star).mean() >= 0.75
