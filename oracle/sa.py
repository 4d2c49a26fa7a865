"""Traditional simulated annealing (serial single-spin Metropolis), the SA baseline of
Section 4.4 and Table 4.  Test infrastructure (see package doc).

Per trial b, independently, one state sigma of N spins of the integer Ising model (h~, J~ at
scale S; H of Eq. 1, H = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i).  Cycle t = 0 .. cycles-1:

* pick one spin i uniformly at random;
* the energy change of flipping it is dE = 2 sigma_i (h_i + sum_j J_ij sigma_j);
* accept the flip if dE <= 0, otherwise with probability exp(-dE / T(t)).

Temperature (Section 4.4): 1/T(t+1) = 1/T(t) + Delta at every cycle, from T_start = 1000 at the
first cycle to T_end = 0.1 at the last.  Energies here are S times the paper's, so the temperature
is S T as well: beta(t) = 1/(S T(t)) = beta_start + t Delta.

Readings where the paper is silent:
* "randomly flips a spin" = one uniformly chosen spin per cycle;
* a flip with dE = 0 is accepted (exp(0) = 1; both clauses of the rule agree);
* first hit: the first t in [0, cycles] at which the state after t cycles has energy E*.

Random stream (Philox4x32-10, key = seed halves; see ``philox``):
* initial spins: counter (i >> 7, 0xFFFFFFFE, 0, b), spin i takes bit (i & 31) of word
  (i & 127) >> 5, bit 1 = +1 (the layout of the annealer's tag-0 draw);
* cycle t: counter (t, 0xFFFFFFFF, 0, b); word 0 picks the spin i = (w0 * N) >> 32, word 1 is
  the acceptance draw: accept iff w1 < 2^32 exp(-dE beta(t)).

The acceptance probability is a floating-point number that decides an integer outcome, so it is
evaluated by ``exp_neg``: an exponential built from a fixed sequence of correctly rounded double
operations (reduction by the nearest multiple of ln 2, the Taylor polynomial of degree 13 in Horner
form, an exact scaling by a power of two).  Any
implementation performing the same operations in the same order takes every decision identically.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from .philox import philox4x32_10

SA_INIT_TAG = 0xFFFFFFFE
SA_STEP_TAG = 0xFFFFFFFF

# ln 2 and 1/ln 2 rounded to double (from 40 digits), and 1/k! for k = 0 .. 13, each rounded once.
_LN2_EXACT = Fraction("0.6931471805599453094172321214581765680755")
_LN2 = float(_LN2_EXACT)
_INV_LN2 = float(1 / _LN2_EXACT)
_TAYLOR = [float(Fraction(1, math.factorial(k))) for k in range(14)]


def exp_neg(x: float) -> float:
    """exp(-x) for x >= 0 by a fixed operation sequence (see module doc); 0 beyond x = 700, so
    that every value stays a normal double and the final scaling by 2^-n is exact.  Relative error
    below 1e-12 over [0, 700]."""
    x = float(x)
    if x > 700.0:
        return 0.0
    n = math.floor(x * _INV_LN2 + 0.5)          # nearest integer to x / ln 2
    r = n * _LN2 - x                            # -(x - n ln 2), |r| <= ln 2 / 2 up to rounding
    p = _TAYLOR[13]
    for k in range(12, -1, -1):
        p = p * r + _TAYLOR[k]
    return math.ldexp(p, -n)


def accept_threshold(de: int, beta: float) -> float:
    """2^32 exp(-dE beta): a flip with dE > 0 is accepted iff the 32-bit draw is below it."""
    return math.ldexp(exp_neg(float(de) * beta), 32)


def sa_schedule(cycles: int, t_start: float = 1000.0, t_end: float = 0.1, scale: int = 12) -> np.ndarray:
    """beta(t) = 1/(S T(t)) for t = 0 .. cycles-1: 1/T grows by the same Delta every cycle
    (Section 4.4), from 1/T_start at t = 0 to 1/T_end at t = cycles - 1."""
    b0 = 1.0 / (scale * t_start)
    b1 = 1.0 / (scale * t_end)
    if cycles == 1:
        return np.array([b0])
    delta = (b1 - b0) / (cycles - 1)
    return np.array([b0 + t * delta for t in range(cycles)])


@dataclass
class SAResult:
    best: np.ndarray          # int64 [T]
    first_hit: np.ndarray     # int64 [T], -1 if E* is never reached
    energy: np.ndarray        # int64 [T]: energy of the final state
    spins: np.ndarray         # int8 [T, N] final state, +-1
    trace: np.ndarray         # int64 [cycles + 1, T]: energy after t cycles


def _energy(h, J, s):
    return -int(h @ s) - int(s @ (J @ s)) // 2


def initial_spins(n: int, b: int, k0: int, k1: int) -> np.ndarray:
    i = np.arange(n)
    words = philox4x32_10(i >> 7, SA_INIT_TAG, 0, b, k0, k1)
    w = np.stack(words)[(i & 127) >> 5, i]
    bits = (w >> (i & 31).astype(np.uint64)) & np.uint64(1)
    return np.where(bits == 1, 1, -1).astype(np.int64)


def sa_anneal(h, J, trials, cycles: int, beta, seed: int, target=None) -> SAResult:
    """Serial Metropolis annealing of every trial in ``trials`` (an int T, or a list of trial
    indices); ``beta`` holds the inverse temperature of each cycle at the integer scale."""
    h = np.asarray(h, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    n = h.shape[0]
    beta = np.asarray(beta, dtype=np.float64)
    assert beta.shape == (cycles,)
    tlist = list(range(trials)) if isinstance(trials, (int, np.integer)) else list(trials)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    T = len(tlist)
    best = np.zeros(T, dtype=np.int64)
    hit = np.full(T, -1, dtype=np.int64)
    energy = np.zeros(T, dtype=np.int64)
    spins = np.zeros((T, n), dtype=np.int8)
    trace = np.zeros((cycles + 1, T), dtype=np.int64)
    steps = np.arange(cycles)
    for col, b in enumerate(tlist):
        s = initial_spins(n, b, k0, k1)
        field = J @ s                               # F_j = sum_k J_jk s_k
        e = _energy(h, J, s)
        w0, w1, _, _ = philox4x32_10(steps, SA_STEP_TAG, 0, b, k0, k1)
        picks = ((w0.astype(np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)
        draws = w1.astype(np.int64)
        best[col] = e
        if target is not None and e == target:
            hit[col] = 0
        trace[0, col] = e
        for t in range(cycles):
            i = int(picks[t])
            de = 2 * int(s[i]) * (int(h[i]) + int(field[i]))
            if de <= 0 or draws[t] < accept_threshold(de, float(beta[t])):
                s[i] = -s[i]
                field += 2 * int(s[i]) * J[:, i]
                e += de
            if e < best[col]:
                best[col] = e
            if target is not None and hit[col] < 0 and e == target:
                hit[col] = t + 1
            trace[t + 1, col] = e
        energy[col] = e
        spins[col] = s
    return SAResult(best=best, first_hit=hit, energy=energy, spins=spins, trace=trace)
