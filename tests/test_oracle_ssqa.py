"""Pins for the oracle's SSQA / SSA sweep, schedules and energies (CPU only)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import gi, metrics, ssqa
from synth import random_gi_pair, random_ising


# ----------------------------------------------------------------------------
# schedules (Section 4.2, Table 2, Table 3; Section 4.4 for SSA)
# ----------------------------------------------------------------------------

def test_jperp_iteration_shape():
    """beta = 3, tau = 100: 400 cycles per iteration, J_perp rises 0 -> 1/6 -> 1/3 -> 1/2
    every 100 cycles, sits at 1/2 for the last tau cycles, then resets."""
    s = ssqa.jperp_schedule(1000, 100, 3, 0, Fraction(1, 2))
    assert s[0] == 0 and s[99] == 0 and s[100] == Fraction(1, 6) and s[200] == Fraction(1, 3)
    assert s[300] == Fraction(1, 2) and s[399] == Fraction(1, 2)
    assert s[400] == 0 and s[700] == Fraction(1, 2) and s[800] == 0 and s[999] == Fraction(1, 6)
    assert max(s) == Fraction(1, 2)
    q = ssqa.scaled(s, 12)
    assert sorted(set(q.tolist())) == [0, 2, 4, 6]


@pytest.mark.parametrize("ec,tau,iters", [(10000, 50, 2), (10000, 100, 1), (20000, 50, 4),
                                          (20000, 100, 2), (40000, 100, 4)])
def test_table3_iteration_counts(ec, tau, iters):
    """Table 3: iterations = EC / R / (tau (beta + 1)) at R = 25; the schedule resets
    J_perp exactly that many times within SC = EC / R cycles."""
    R, beta = 25, 3
    assert metrics.iterations(ec, R, tau, beta) == iters
    sc = ec // R
    s = ssqa.jperp_schedule(sc, tau, beta, 0, Fraction(1, 2))
    starts = sum(1 for t in range(sc) if t % (tau * (beta + 1)) == 0)
    assert starts == iters


def test_equivalent_cycles():
    """Eq. 9 example: EC = 20,000 gives SC = 2,000 at R = 10 and 500 at R = 40."""
    assert metrics.equivalent_cycles(10, 2000) == 20000
    assert metrics.equivalent_cycles(40, 500) == 20000


def test_ssa_i0_schedule():
    """Section 4.4: I_0 = 1, 2, 4, 8, 16 for tau = 10 cycles each (beta = 0.5),
    50 cycles per iteration, then back to 1."""
    s = ssqa.ssa_i0_schedule(120, 10, Fraction(1, 2), 1, 16)
    assert [s[t] for t in (0, 9, 10, 20, 30, 40, 49, 50, 60, 100)] == [1, 1, 2, 4, 8, 16, 16, 1, 2, 1]


def test_scaled_rejects_inexact():
    with pytest.raises(ValueError):
        ssqa.scaled([Fraction(1, 6)], 4)


# ----------------------------------------------------------------------------
# the update rule, hand-computed
# ----------------------------------------------------------------------------

def test_step_hand_computed_two_spins_two_replicas():
    """h = (5, -3), J01 = 2, alpha = 1, I0 = 4, n_rnd = 2, J_perp = 3, d = 1.
    Is(t) = [[1, -2], [-4, 3]] -> sigma(t) = [[+1, -1], [-1, +1]];
    sigma(t-1) = [[+1, +1], [-1, -1]]; r = [[+1, -1], [-1, +1]].
    Replica 0: F = (-2, 2); coupling 3 sigma_{.,1}(t-1) = (-3, -3);
      I = (5-2+2-3, -3+2-2-3) = (2, -6); s = (3, -8) -> Is = (3, -4).
    Replica 1: F = (2, -2); coupling 3 sigma_{.,0}(t-1) = (3, 3);
      I = (5+2-2+3, -3-2+2+3) = (8, 0); s = (4, 3) -> Is = (3, 3) (s = 4 >= I0 saturates to I0 - alpha)."""
    h = np.array([5, -3])
    J = np.array([[0, 2], [2, 0]])
    Is = np.array([[[1, -2], [-4, 3]]])
    sigma_t = np.where(Is >= 0, 1, -1)
    sigma_d = np.array([[[1, 1], [-1, -1]]])
    r = np.array([[[1, -1], [-1, 1]]])
    F = ssqa.field(J, sigma_t)
    assert F.tolist() == [[[-2, 2], [2, -2]]]
    Is1, s1 = ssqa.ssqa_step(Is, F, sigma_d, h, r, 3, 4, 1, 2, 0)
    assert Is1.tolist() == [[[3, -4], [3, 3]]]
    assert s1.tolist() == [[[1, -1], [1, 1]]]


def test_step_coupling_direction_three_replicas():
    """One spin, R = 3, h = J = 0, no noise, J_perp = 2, Is = 0, sigma(t-d) = (+1, -1, -1).
    Mode 0 (upper replica only, Eq. 6a): coupling = 2 * (sigma_1, sigma_2, sigma_0) = (-2, -2, 2).
    Mode 1 (both neighbours): adds 2 * (sigma_2, sigma_0, sigma_1) -> (-4, 0, 0)."""
    h = np.array([0])
    Is = np.zeros((1, 3, 1), dtype=np.int64)
    F = np.zeros_like(Is)
    sd = np.array([1, -1, -1]).reshape(1, 3, 1)
    r = np.ones_like(Is)
    Is0, s0 = ssqa.ssqa_step(Is, F, sd, h, r, 2, 10, 1, 0, 0)
    assert Is0.ravel().tolist() == [-2, -2, 2] and s0.ravel().tolist() == [-1, -1, 1]
    Is1, s1 = ssqa.ssqa_step(Is, F, sd, h, r, 2, 10, 1, 0, 1)
    assert Is1.ravel().tolist() == [-4, 0, 0] and s1.ravel().tolist() == [-1, 1, 1]


def test_counter_tie_breaks():
    """Eq. 6b/6c boundaries with I0 = 5, alpha = 1: s = 5 -> 4; s = 4 -> 4; s = -5 -> -5;
    s = -6 -> -5; s = 0 -> 0 with sigma = +1; s = -1 -> -1 with sigma = -1."""
    Is = np.zeros(6, dtype=np.int64)
    I = np.array([5, 4, -5, -6, 0, -1])
    Is1, s1 = ssqa.counter_update(Is, I, 5, 1)
    assert Is1.tolist() == [4, 4, -5, -5, 0, -1]
    assert s1.tolist() == [1, 1, -1, -1, 1, -1]


def test_anneal_hand_computed_trace():
    """Two cycles of the two-spin, two-replica model without noise, from a given
    state (d = 1).  Worked by hand:
      t=0: sigma = [[+1,-1],[-1,+1]], E = (-6, 10);
           I = [[0,-4],[10,-2]], Is(1) = [[1,-4],[3,1]], sigma(1) = [[+1,-1],[+1,+1]]
      t=1: E = (-6, -4); coupling from sigma(0): [[-3,3],[3,-3]];
           I = [[0,2],[10,-4]], Is(2) = [[1,-2],[3,-3]], sigma(2) = [[+1,-1],[+1,-1]]
      t=2: E = (-6, -6).  The ground energy of this model is -6 (state (+1,-1))."""
    h = np.array([5, -3])
    J = np.array([[0, 2], [2, 0]])
    Is0 = np.array([[[1, -2], [-4, 3]]])
    s0 = np.array([[[1, -1], [-1, 1]]])
    sm1 = np.array([[[1, 1], [-1, -1]]])
    st = ssqa.AnnealState(cycle=0, Is=Is0, history=[s0, sm1])
    res = ssqa.anneal(h, J, 2, [0], 2, [3, 3], [4, 4], alpha=1, n_rnd=0, delay=1, seed=0,
                      coupling_mode=0, target=-6, state=st)
    assert res.energy[:, 0, :].tolist() == [[-6, 10], [-6, -4], [-6, -6]]
    assert res.Is.tolist() == [[[1, -2], [3, -3]]]
    assert res.best.tolist() == [-6] and res.first_hit.tolist() == [0]
    assert res.state.history[1].tolist() == [[[1, -1], [1, 1]]]


# ----------------------------------------------------------------------------
# energies
# ----------------------------------------------------------------------------

def test_energy_from_field_equals_direct_double_sum():
    h, J = random_ising(37, seed=5, h_max=50, j_max=9)
    rng = np.random.default_rng(1)
    sig = rng.choice([-1, 1], size=(6, 37))
    F = ssqa.field(J, sig)
    e = ssqa.energy_from_field(h, sig, F)
    assert [ssqa.energy_direct(h, J, s) for s in sig] == e.tolist()


def test_qmc_energy_reduces_to_sum_of_problem_energies():
    """Eq. 4 with J_perp = 0 is the sum of the replicas' H_p; with identical replicas
    the coupling term is -J_perp R N."""
    h, J = random_ising(9, seed=2)
    rng = np.random.default_rng(3)
    sig = rng.choice([-1, 1], size=(2, 4, 9))
    hp = [[ssqa.energy_direct(h, J, sig[b, k]) for k in range(4)] for b in range(2)]
    assert ssqa.qmc_energy(h, J, sig, 0).tolist() == [sum(x) for x in hp]
    same = np.repeat(sig[:, :1], 4, axis=1)
    e0 = [4 * ssqa.energy_direct(h, J, same[b, 0]) for b in range(2)]
    assert ssqa.qmc_energy(h, J, same, 5).tolist() == [e - 5 * 4 * 9 for e in e0]


# ----------------------------------------------------------------------------
# special cases and invariants of a full anneal
# ----------------------------------------------------------------------------

def _gi_model(n, seed, scale=12):
    pair = random_gi_pair(n, 0.5, seed)
    return gi.gi_ising(pair.a1, pair.a2, scale)


def test_invariants_counter_range_and_sign():
    h, J, e_star = _gi_model(4, 1)
    SC = 60
    q = ssqa.scaled(ssqa.jperp_schedule(SC, 5, 3, 0, Fraction(1, 2)), 12)
    i0 = np.full(SC, 24)
    state = None
    for _ in range(3):
        res = ssqa.anneal(h, J, 5, 3, 20, q, i0, 1, 12, 1, seed=11, target=e_star, state=state)
        state = res.state
        assert res.Is.min() >= -24 and res.Is.max() <= 23
        assert np.array_equal(res.sigma, np.where(res.Is >= 0, 1, -1))
        assert (res.best >= e_star).all()


def test_decoupled_replicas_equal_independent_ssa_chains():
    """J_perp = 0: the R replicas decouple and each follows SSA (Eq. 2) with constant
    I_0 on the same random-stream positions."""
    h, J = random_ising(40, seed=9, h_max=30, j_max=5)
    SC, R = 30, 4
    q = np.zeros(SC, dtype=np.int64)
    i0 = np.full(SC, 20)
    res = ssqa.anneal(h, J, R, [0, 3], SC, q, i0, 1, 9, 1, seed=21)
    e_ssa, Is_ssa, s_ssa = ssqa.ssa_anneal(h, J, [0, 3], SC, i0, 1, 9, seed=21, chains=range(R))
    assert np.array_equal(res.energy, e_ssa)
    assert np.array_equal(res.Is, Is_ssa)


def test_hopfield_special_case():
    """n_rnd = 0, J_perp = 0, I_0 = alpha = 1 and fields never zero (odd h, even J):
    the counter lives in {-1, 0} and the update is the synchronous threshold network
    sigma(t+1) = sgn(h + J sigma(t)); with symmetric J it ends in a fixed point or a
    2-cycle (Goles-Fogelman-Pellegrin)."""
    rng = np.random.default_rng(4)
    N = 30
    h = 2 * rng.integers(-5, 6, size=N) + 1
    A = rng.integers(-3, 4, size=(N, N))
    J = 2 * np.triu(A, 1)
    J = J + J.T
    SC = 200
    res = ssqa.anneal(h, J, 1, 3, SC, np.zeros(SC, int), np.ones(SC, int), 1, 0, 0, seed=5)
    assert set(np.unique(res.Is).tolist()) <= {-1, 0}
    # replay with the threshold map from the same initial spins
    st = ssqa.initial_state(N, 1, np.arange(3), 5, 1, 0)
    sig = st.history[0][:, 0, :].copy()
    traj = [sig]
    for _ in range(SC):
        sig = np.where(h + sig @ J.T > 0, 1, -1)
        traj.append(sig)
    assert np.array_equal(traj[-1], res.sigma[:, 0, :])
    assert np.array_equal(traj[-1], traj[-3])


def test_one_cycle_against_scalar_loops():
    """The vectorised cycle against an element-by-element evaluation of Eq. 6 (indices
    b, k, i written out), for both coupling modes and d = 0, 1, 2."""
    from oracle.philox import stream_signs
    h, J = random_ising(11, seed=3, h_max=20, j_max=4)
    R, B = 3, 2
    for mode in (0, 1):
        for d in (0, 1, 2):
            SC = 4
            q = np.array([3, 5, 7, 9])
            i0 = np.array([15, 16, 17, 18])
            res = ssqa.anneal(h, J, R, B, SC, q, i0, 2, 6, d, seed=8, coupling_mode=mode)
            # recompute by scalar loops from the initial state
            st = ssqa.initial_state(11, R, np.arange(B), 8, 2, d)
            Is = st.Is.copy()
            hist = list(st.history)
            for t in range(SC):
                sig = hist[0]
                r = stream_signs(8, t + 1, 11, R, B)
                new_Is = np.zeros_like(Is)
                for b in range(B):
                    for k in range(R):
                        for i in range(11):
                            f = sum(int(J[i, j]) * int(sig[b, k, j]) for j in range(11))
                            c = q[t] * hist[d][b, (k + 1) % R, i]
                            if mode == 1:
                                c += q[t] * hist[d][b, (k - 1) % R, i]
                            s = Is[b, k, i] + h[i] + f + 6 * r[b, k, i] + c
                            if s >= i0[t]:
                                new_Is[b, k, i] = i0[t] - 2
                            elif s < -i0[t]:
                                new_Is[b, k, i] = -i0[t]
                            else:
                                new_Is[b, k, i] = s
                Is = new_Is
                hist = [np.where(Is >= 0, 1, -1)] + hist[:d]
            assert np.array_equal(Is, res.Is)


def test_trial_subset_and_resume_are_exact():
    """Trials are independent (a subset replays exactly) and an anneal split at any
    cycle and resumed from its saved state equals the uninterrupted run."""
    h, J, e_star = _gi_model(3, 2)
    SC = 80
    q = ssqa.scaled(ssqa.jperp_schedule(SC, 10, 3, 0, Fraction(1, 2)), 12)
    i0 = np.full(SC, 24)
    full = ssqa.anneal(h, J, 4, 6, SC, q, i0, 1, 12, 1, seed=3, target=e_star)
    sub = ssqa.anneal(h, J, 4, [1, 5], SC, q, i0, 1, 12, 1, seed=3, target=e_star)
    assert np.array_equal(full.energy[:, [1, 5]], sub.energy)
    assert np.array_equal(full.first_hit[[1, 5]], sub.first_hit)
    a = ssqa.anneal(h, J, 4, 6, 33, q, i0, 1, 12, 1, seed=3, target=e_star)
    b = ssqa.anneal(h, J, 4, 6, SC - 33, q, i0, 1, 12, 1, seed=3, target=e_star, state=a.state)
    assert np.array_equal(np.concatenate([a.energy, b.energy[1:]]), full.energy)
    assert np.array_equal(b.Is, full.Is)


@pytest.mark.parametrize("n,trials,min_ps", [(5, 20, 0.9), (10, 10, 0.7)])
def test_small_gi_instances_are_solved(n, trials, min_ps):
    """Statistical sanity, not parity: with the paper's SSQA parameters (Table 2,
    R = 25, SC = 1600, tau = 100) Table 4 reports P_s = 100 % for N = 25 and 100.
    Our instances and random streams differ, so only a high P_s is required."""
    h, J, e_star = _gi_model(n, 100 + n)
    SC, R = 1600, 25
    q = ssqa.scaled(ssqa.jperp_schedule(SC, 100, 3, 0, Fraction(1, 2)), 12)
    i0 = np.full(SC, 24)
    res = ssqa.anneal(h, J, R, trials, SC, q, i0, 1, 12, 1, seed=1, target=e_star)
    ps = metrics.success_probability(res.best, e_star)
    assert ps >= min_ps, ps
