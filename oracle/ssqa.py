"""SSQA and SSA sweeps in exact integer arithmetic.  Test infrastructure.

State per trial b: R replicas of N spins.  Arrays are indexed [b, k, i]
(trial, replica, spin).  The Ising model is given at an integer scale S (h~,
J~ int, J~ symmetric with zero diagonal); the noise amplitude n_rnd, the
replica coupling J_perp(t), the bound I_0(t) and alpha are integers at the
same scale.

SSQA update of spin i in replica k for t -> t+1 (Eq. 6a-c, Section 3.2):
    I   = h_i + sum_j J_ij sigma_{j,k}(t) + n_rnd r_{i,k}(t) + J_perp(t) sigma_{i,k+1}(t-d)
    s   = Is_{i,k}(t) + I
    Is_{i,k}(t+1) = I_0 - alpha  if s >= I_0
                    -I_0         else if s < -I_0
                    s            otherwise
    sigma_{i,k}(t+1) = +1 if Is_{i,k}(t+1) >= 0 else -1
All N*R spins of a trial are updated together from the state at t (Section
3.2: the spins are updated in parallel).  Replica k+1 wraps to replica 0: the
top replica is coupled to the bottom one (Fig. 2, Section 3.1).

Readings where the paper is silent or ambiguous:
* coupling_mode 0 uses only the upper replica k+1, as Eq. 6a is printed;
  coupling_mode 1 adds the lower replica k-1 as well (the replica network of
  Fig. 2 is coupled both ways).
* the delayed spin sigma(t-d) for t < d is the initial state sigma(0).
* initial state: sigma(0) is drawn from the random stream (tag 0) and
  Is(0) = 0 for sigma = +1, -alpha for sigma = -1, so that sigma(0) = sign(Is(0)).
  Neither spins nor counters are reset between iterations; only J_perp is.
* the noise r is drawn per spin, replica, trial and cycle (see ``philox``).

SSA (Eq. 2a-c, Section 2.2) is the same counter without replicas or coupling.
"""

from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .philox import stream_signs


# ----------------------------------------------------------------------------
# schedules
# ----------------------------------------------------------------------------

def jperp_schedule(cycles: int, tau: int, beta: int, jmin, jmax) -> list[Fraction]:
    """J_perp(t) for t = 0 .. cycles-1 (Section 4.2, Table 2).

    Each iteration lasts tau * (beta + 1) cycles.  J_perp starts an iteration at
    jmin and grows by (jmax - jmin) / beta every tau cycles, so its last tau cycles
    sit at jmax; the next iteration starts again from jmin.
    """
    jmin, jmax = Fraction(jmin), Fraction(jmax)
    step = (jmax - jmin) / beta
    out = []
    j = jmin
    for t in range(cycles):
        if t % (tau * (beta + 1)) == 0:
            j = jmin                          # a new iteration resets J_perp
        elif t % tau == 0:
            j = j + step                      # raised every tau cycles
        out.append(j)
    return out


def ssa_i0_schedule(cycles: int, tau: int, beta, i0_min, i0_max) -> list[Fraction]:
    """I_0(t) of SSA (Section 4.4): starts at I_0min and is multiplied by 1/beta
    every tau cycles up to I_0max; after tau cycles at I_0max the next iteration
    starts again from I_0min."""
    beta, i0_min, i0_max = Fraction(beta), Fraction(i0_min), Fraction(i0_max)
    out = []
    i0 = i0_min
    since = 0
    for t in range(cycles):
        if t > 0 and since == tau:
            since = 0
            i0 = i0_min if i0 >= i0_max else min(i0 / beta, i0_max)
        out.append(i0)
        since += 1
    return out


def scaled(values, scale: int) -> np.ndarray:
    """values * S as exact int64; raises if any product is not an integer."""
    out = []
    for v in values:
        f = Fraction(v) * scale
        if f.denominator != 1:
            raise ValueError(f"{v} * {scale} is not an integer")
        out.append(int(f))
    return np.asarray(out, dtype=np.int64)


# ----------------------------------------------------------------------------
# energies
# ----------------------------------------------------------------------------

def field(J: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """F[..., i] = sum_j J_ij sigma[..., j], exact (float64 product of small integers;
    J may be passed already converted to float64)."""
    shp = sigma.shape
    s2 = sigma.reshape(-1, shp[-1]).astype(np.float64)
    Jf = J if J.dtype == np.float64 else J.astype(np.float64)
    F = s2 @ Jf.T
    return np.rint(F).astype(np.int64).reshape(shp)


def energy_from_field(h: np.ndarray, sigma: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Problem Hamiltonian (Eq. 1 / Eq. 5) from the field F = J sigma:
    H = -sum_i h_i sigma_i - (1/2) sum_i sigma_i F_i  (J symmetric, zero diagonal)."""
    two_e = -2 * (sigma * h).sum(-1) - (sigma * F).sum(-1)
    return two_e // 2


def energy_direct(h: np.ndarray, J: np.ndarray, sigma: np.ndarray) -> int:
    """Eq. 1 as printed: -sum_i h_i sigma_i - sum_{i<j} J_ij sigma_i sigma_j (one state)."""
    s = np.asarray(sigma, dtype=np.int64)
    N = len(s)
    e = 0
    for i in range(N):
        e -= int(h[i]) * int(s[i])
        for j in range(i + 1, N):
            e -= int(J[i, j]) * int(s[i]) * int(s[j])
    return e


def qmc_energy(h: np.ndarray, J: np.ndarray, sigma: np.ndarray, jperp: int) -> np.ndarray:
    """QMC Hamiltonian H_c (Eq. 4) of each trial: sum over replicas of H_p minus
    J_perp sum_i sigma_{i,k} sigma_{i,k+1}, replica R wrapping to replica 1.
    sigma is [B, R, N]; returns [B]."""
    F = field(J, sigma)
    hp = energy_from_field(h, sigma, F).sum(-1)
    R = sigma.shape[-2]
    up = sigma[..., (np.arange(R) + 1) % R, :]
    return hp - jperp * (sigma * up).sum((-1, -2))


# ----------------------------------------------------------------------------
# one update
# ----------------------------------------------------------------------------

def counter_update(Is: np.ndarray, I: np.ndarray, i0: int, alpha: int):
    """Eq. 6b / Eq. 2b (saturating integral counter) and Eq. 6c / Eq. 2c (sign)."""
    s = Is + I
    Is_next = np.where(s >= i0, i0 - alpha, np.where(s < -i0, -i0, s))
    sigma_next = np.where(Is_next >= 0, 1, -1)
    return Is_next.astype(np.int64), sigma_next.astype(np.int64)


def ssqa_step(Is, F, sigma_delayed, h, r, jperp_t: int, i0_t: int, alpha: int, n_rnd: int,
              coupling_mode: int = 0):
    """One synchronous SSQA update of every spin and replica (Eq. 6a-c).

    Is, F, sigma_delayed, r: int arrays [..., R, N]; F = J sigma(t) per replica;
    sigma_delayed = sigma(t - d); r = +-1 noise.  Returns (Is(t+1), sigma(t+1)).
    """
    R = Is.shape[-2]
    upper = sigma_delayed[..., (np.arange(R) + 1) % R, :]        # sigma_{i,k+1}(t-d)
    coupling = jperp_t * upper
    if coupling_mode == 1:
        lower = sigma_delayed[..., (np.arange(R) - 1) % R, :]    # sigma_{i,k-1}(t-d)
        coupling = coupling + jperp_t * lower
    I = h + F + n_rnd * r + coupling                              # Eq. 6a
    return counter_update(Is, I, i0_t, alpha)


def ssa_step(Is, F, h, r, i0_t: int, alpha: int, n_rnd: int):
    """One synchronous SSA update (Eq. 2a-c)."""
    I = h + F + n_rnd * r                                         # Eq. 2a
    return counter_update(Is, I, i0_t, alpha)


# ----------------------------------------------------------------------------
# full anneal
# ----------------------------------------------------------------------------

@dataclass
class AnnealState:
    """Everything needed to continue an anneal at cycle ``cycle``: the counters
    Is(t) and the spin history sigma(t), sigma(t-1), ..., sigma(t-d)."""
    cycle: int
    Is: np.ndarray
    history: list


@dataclass
class AnnealResult:
    energy: np.ndarray        # [cycles+1, B, R]: H_p of every replica at t = start .. start+cycles
    best: np.ndarray          # [B] min over replicas and time
    first_hit: np.ndarray     # [B] first t (absolute) with some replica at the target, -1 if none
    state: AnnealState        # final state
    trials: np.ndarray        # trial indices b simulated

    @property
    def Is(self):
        return self.state.Is

    @property
    def sigma(self):
        return self.state.history[0]


def initial_state(N: int, replicas: int, trial_ids, seed: int, alpha: int, delay: int) -> AnnealState:
    sigma0 = stream_signs(seed, 0, N, replicas, trial_ids)       # tag 0
    Is0 = np.where(sigma0 > 0, 0, -alpha).astype(np.int64)
    return AnnealState(cycle=0, Is=Is0, history=[sigma0] * (delay + 1))


def anneal(h, J, replicas: int, trials, cycles: int, jperp_sched, i0_sched, alpha: int,
           n_rnd: int, delay: int, seed: int, coupling_mode: int = 0, target=None,
           state: AnnealState | None = None) -> AnnealResult:
    """Run SSQA for ``cycles`` cycles.

    trials: a count T (trials 0..T-1) or a sequence of trial indices; trials are
    independent, so any subset reproduces those trials of a larger run exactly.
    jperp_sched, i0_sched: integer arrays indexed by absolute cycle t.
    state: resume from a saved AnnealState (its cycle gives the start t).
    The energy of every replica is recorded for t = start .. start + cycles,
    including the state after the last update (one more field evaluation).
    """
    h = np.asarray(h, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    Jf = J.astype(np.float64)
    N = len(h)
    trial_ids = np.arange(trials) if np.isscalar(trials) else np.asarray(trials)
    if state is None:
        state = initial_state(N, replicas, trial_ids, seed, alpha, delay)
    t0 = state.cycle
    Is = state.Is.copy()
    hist = list(state.history)
    assert len(hist) == delay + 1
    energies = []
    for t in range(t0, t0 + cycles + 1):
        sigma = hist[0]
        F = field(Jf, sigma)
        energies.append(energy_from_field(h, sigma, F))
        if t == t0 + cycles:
            break
        r = stream_signs(seed, t + 1, N, replicas, trial_ids)    # tag t+1
        Is, sigma_next = ssqa_step(Is, F, hist[delay], h, r, int(jperp_sched[t]), int(i0_sched[t]),
                                   alpha, n_rnd, coupling_mode)
        hist = [sigma_next] + hist[:delay]
    energy = np.stack(energies)                                   # [cycles+1, B, R]
    best = energy.min(axis=(0, 2))
    first_hit = np.full(len(trial_ids), -1, dtype=np.int64)
    if target is not None:
        hit = (energy.min(axis=2) == target)                      # [cycles+1, B]
        any_hit = hit.any(axis=0)
        first_hit[any_hit] = t0 + hit.argmax(axis=0)[any_hit]
    return AnnealResult(energy=energy, best=best, first_hit=first_hit,
                        state=AnnealState(cycle=t0 + cycles, Is=Is, history=hist),
                        trials=trial_ids)


def ssa_anneal(h, J, trials, cycles: int, i0_sched, alpha: int, n_rnd: int, seed: int,
               chains=(0,)):
    """SSA (Eq. 2a-c) on independent chains.  Chain k of trial b draws its spins and
    noise from the same stream positions (tag, i >> 7, k, b) as replica k of SSQA.
    Returns (energy [cycles+1, B, K], Is, sigma)."""
    h = np.asarray(h, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    N = len(h)
    trial_ids = np.arange(trials) if np.isscalar(trials) else np.asarray(trials)
    chains = np.asarray(chains)
    sigma = stream_signs(seed, 0, N, chains, trial_ids)
    Is = np.where(sigma > 0, 0, -alpha).astype(np.int64)
    energies = []
    for t in range(cycles + 1):
        F = field(J, sigma)
        energies.append(energy_from_field(h, sigma, F))
        if t == cycles:
            break
        r = stream_signs(seed, t + 1, N, chains, trial_ids)
        Is, sigma = ssa_step(Is, F, h, r, int(i0_sched[t]), alpha, n_rnd)
    return np.stack(energies), Is, sigma
