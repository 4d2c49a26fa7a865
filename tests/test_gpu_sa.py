"""GPU parity of the SA baseline (serial single-spin Metropolis, Section 4.4): the many-chain HIP kernel
against the oracle, bit for bit, through the C ABI."""

import sys

import numpy as np
import pytest

from oracle import gi, sa
from synth import random_ising
from tests.parity_util import gi_case

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2302_12454_amd as lib
    return lib


def _run(lib, h, J, trials, beta, seed, target=None, trace=False):
    import torch
    res = lib.ssqa_sa_anneal(lib.Problem(h, J), trials=trials, beta=beta, seed=seed, target=target, trace=trace)
    torch.cuda.synchronize()
    out = {k: getattr(res, k).cpu().numpy() for k in ("best_energy", "first_hit", "final_energy", "final_spins")}
    out["trace"] = res.energy_trace.cpu().numpy() if trace else None
    return out


def _same(g, ref, cols=None):
    sel = slice(None) if cols is None else np.asarray(cols)
    assert np.array_equal(g["best_energy"][sel], ref.best)
    assert np.array_equal(g["first_hit"][sel], ref.first_hit)
    assert np.array_equal(g["final_energy"][sel], ref.energy)
    assert np.array_equal(g["final_spins"][sel], ref.spins)
    if g["trace"] is not None:
        tr = g["trace"][:, sel]
        if not np.array_equal(tr, ref.trace):
            bad = np.argwhere(tr != ref.trace)
            raise AssertionError(f"trace differs at {len(bad)} entries, first {bad[0].tolist()}")


def test_sa_gi_n5_table4_config(lib):
    """N = 25 GI, the Table 4 SA configuration (40,000 cycles, T 1000 -> 0.1), 16 chains."""
    _note("case SA gi5 N=25 T=16 cycles=40000")
    h, J, e_star = gi_case(5, 0)
    beta = sa.sa_schedule(40000, 1000.0, 0.1, 12)
    g = _run(lib, h, J, 16, beta, 3, target=e_star)
    _same(g, sa.sa_anneal(h, J, 16, 40000, beta, 3, target=e_star))
    assert (g["best_energy"] == e_star).mean() > 0.7


@pytest.mark.parametrize("n,trials,cycles,j_max,seed", [
    (300, 9, 3000, 9, 1),      # ragged tiles (300 of 384 rows), one int8 plane, full trace
    (70, 6, 2000, 300, 2),     # two int8 planes
    (1, 3, 50, 1, 3),          # a single spin
    (129, 5, 1500, 12, 4),     # one row past a tile
])
def test_sa_random_ising_full_trace(lib, n, trials, cycles, j_max, seed):
    _note(f"case SA random n={n} T={trials} cycles={cycles}")
    h, J = random_ising(n, seed, h_max=80, j_max=j_max)
    beta = sa.sa_schedule(cycles, 200.0, 0.5, 12)
    g = _run(lib, h, J, trials, beta, seed, trace=True)
    _same(g, sa.sa_anneal(h, J, trials, cycles, beta, seed))


def test_sa_temperature_limits(lib):
    """beta = 0 accepts every proposal; a huge beta accepts only dE <= 0 (0 threshold beyond x = 700)."""
    _note("case SA beta limits")
    h, J = random_ising(50, 6, h_max=40, j_max=7)
    for beta_value in (0.0, 1e300):
        beta = np.full(800, beta_value)
        g = _run(lib, h, J, 4, beta, 9, trace=True)
        _same(g, sa.sa_anneal(h, J, 4, 800, beta, 9))


def test_sa_gi50_sampled_chains(lib):
    """N = 2500 GI at the Table 4 configuration (100 chains, 40,000 cycles): chains 0 and 99 replayed by
    the oracle; every chain's final energy equals Eq. 1 of its final state and best >= E*."""
    _note("case SA gi50 N=2500 T=100 cycles=40000 (sampled)")
    h, J, e_star = gi_case(50, 2)
    beta = sa.sa_schedule(40000, 1000.0, 0.1, 12)
    g = _run(lib, h, J, 100, beta, 5, target=e_star)
    _same(g, sa.sa_anneal(h, J, [0, 99], 40000, beta, 5, target=e_star), cols=[0, 99])
    s = g["final_spins"].astype(np.int64)
    direct = -(s @ h) - np.einsum("ti,ti->t", s, s @ J.astype(np.int64)) // 2
    assert np.array_equal(direct, g["final_energy"])
    assert (g["best_energy"] >= e_star).all()


def test_sa_large_n_fewer_chains_per_group(lib):
    """N = 8300 (padded 8320): a chain's fields and spins take 41.6 KB of LDS, so three chains share a
    workgroup; sampled against the oracle."""
    _note("case SA large N=8300 T=5 cycles=300")
    h, J = random_ising(8300, 12, h_max=30, j_max=3, density=0.2)
    beta = sa.sa_schedule(300, 50.0, 1.0, 12)
    g = _run(lib, h, J, 5, beta, 8, trace=True)
    _same(g, sa.sa_anneal(h, J, 5, 300, beta, 8))


def test_sa_rejects_bad_beta(lib):
    h, J = random_ising(10, 1, h_max=5, j_max=3)
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_sa_anneal(lib.Problem(h, J), trials=2, beta=np.array([0.1, -1.0]), seed=0)
    assert ei.value.name == "SSQA_EINVAL"
