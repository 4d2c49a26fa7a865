"""Pins for the oracle's time-to-solution (Eq. 10) against Table 4 (CPU only)."""

import json
import math
import os

import pytest

from oracle import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table4_comparison.json")


def _rows():
    with open(GOLDEN) as f:
        g = json.load(f)
    return g["rows"], g["p_target"], g["claims"]


def test_tts_reproduces_every_printed_value():
    """Eq. 10 applied to Table 4's own P_s and t gives its printed TTS: within the
    interval implied by the printed rounding of P_s (whole percent) and t, and within
    2 % of the point value."""
    rows, pt, _ = _rows()
    checked = 0
    for N, method, ps, t, tts in rows:
        if ps == "na":
            continue
        if tts == "approx0":
            assert ps == 100 and metrics.tts(t, 1.0, pt) == 0.0
            continue
        if tts is None:
            assert ps == 0 and metrics.tts(t, 0.0, pt) is None
            continue
        point = metrics.tts(t, ps / 100, pt)
        assert abs(point - tts) / tts < 0.02, (N, method, point, tts)
        lo = metrics.tts(t * 0.995, min(ps + 0.5, 99.99) / 100, pt)
        hi = metrics.tts(t * 1.005, (ps - 0.5) / 100, pt)
        assert lo <= tts <= hi, (N, method, lo, tts, hi)
        checked += 1
    assert checked == 10


def test_tts_reduction_claim():
    """SSQA reduces TTS by 91.4 % relative to SSA at N = 2025 (Section 4.4)."""
    rows, pt, claims = _rows()
    d = {(r[0], r[1]): r for r in rows}
    red = 100 * (1 - d[(2025, "SSQA")][4] / d[(2025, "SSA")][4])
    assert round(red, 1) == claims["ssqa_vs_ssa_tts_reduction_percent_at_N2025"]


def test_tts_edges_and_monotonicity():
    assert metrics.tts(2.0, 1.0) == 0.0
    assert metrics.tts(2.0, 0.0) is None
    assert metrics.tts(1.0, 0.5) == pytest.approx(math.log(0.01) / math.log(0.5))
    assert metrics.tts(1.0, 0.9) < metrics.tts(1.0, 0.5) < metrics.tts(1.0, 0.1)
