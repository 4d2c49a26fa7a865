"""Success probability, time-to-solution and equivalent cycles.  Test infrastructure.

* P_s(t): the fraction of trials that reach the global minimum energy within the
  run (Section 4.3; 100 trials in the paper, Section 4.4).
* TTS = t ln(1 - P_T) / ln(1 - P_s(t))  (Eq. 10), P_T = 0.99 in the paper.
  P_s = 1 gives a denominator of minus infinity, i.e. TTS -> 0 (printed as
  "approx. 0" in Table 4); P_s = 0 leaves TTS undefined (returned as None).
* EC = R x SC  (Eq. 9).
"""

from __future__ import annotations

import math

import numpy as np


def success_probability(best: np.ndarray, target: int) -> float:
    best = np.asarray(best)
    return float((best == target).mean()) if best.size else 0.0


def tts(t: float, p_s: float, p_target: float = 0.99):
    """Eq. 10.  Returns 0.0 for p_s >= 1 and None for p_s <= 0."""
    if p_s >= 1.0:
        return 0.0
    if p_s <= 0.0:
        return None
    return t * math.log(1.0 - p_target) / math.log(1.0 - p_s)


def equivalent_cycles(replicas: int, cycles: int) -> int:
    return replicas * cycles


def iterations(ec: int, replicas: int, tau: int, beta: int) -> float:
    """Number of J_perp iterations, EC / R / (tau (beta + 1)) (Table 2, Table 3)."""
    return ec / replicas / (tau * (beta + 1))
