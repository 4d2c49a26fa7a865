"""GPU tests of the row-split form of a plain anneal (ssqa_anneal with split_rows): every trial's rows spread
over row groups of workgroups, one launch per cycle.  Forced (split_rows = 1) it gives the persistent form's
results (split_rows = -1) bit for bit (best, first hit, energy trace, final counters) for both operand types,
delays 0 to 2, both coupling modes, the general epilogue, 32- and 64-column blocks, zero cycles and groups of
one tile whose K steps the workgroup's four waves share (partial sums added through LDS); on small cases both
forms equal the oracle, SSA's (R = 1, Eq. 2) included.  An SSA-shaped anneal (N = 2500, R = 1) left to the
automatic choice equals both forced forms, and Table 4's SSA and SSQA shapes at N = 2500 equal the oracle
over hundreds of split launches."""

import sys
from fractions import Fraction

import numpy as np
import pytest

from oracle import ssqa
from synth import random_ising
from tests.parity_util import assert_same, gi_case, paper_schedules, run_gpu, run_oracle

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


def _same(a, b):
    for key in a:
        if a[key] is None:
            assert b[key] is None
            continue
        if not np.array_equal(a[key], b[key]):
            bad = np.argwhere(a[key] != b[key])
            raise AssertionError(f"{key} differs at {len(bad)} entries, first {bad[0].tolist()}")


@pytest.mark.parametrize("n,R,T,SC,delay,mode,alpha,j_max,bc", [
    (700, 8, 10, 30, 1, 0, 1, 4, 32),      # fp4, 6 tiles in 2 row groups, 3 column blocks
    (900, 4, 40, 25, 2, 1, 3, 60, 64),     # int8, d = 2, both neighbours, general epilogue
    (1300, 1, 100, 40, 0, 0, 1, 4, 64),    # SSA-shaped: R = 1, d = 0, 11 tiles (last group of 3)
    (300, 16, 7, 20, 1, 1, 2, 30, 32),     # 3 tiles in one group, alpha = 2, int8
    (520, 32, 3, 0, 1, 0, 1, 4, 64),       # zero cycles: sigma(0)'s energy only
    (1100, 2, 20, 12, 1, 1, 3, 300, 32),   # int8 on two planes, the four waves sharing each tile's 18 K steps
    (1900, 4, 16, 10, 2, 0, 1, 4, 32),     # fp4 at the fewest K steps the waves share (16), d = 2
    (2100, 1, 40, 8, 0, 1, 1, 4, 32),      # fp4, 24 K steps over the waves, d = 0, both neighbours
])
def test_forced_split_equals_persistent(lib, n, R, T, SC, delay, mode, alpha, j_max, bc):
    _note(f"case split anneal n={n} R={R} T={T} SC={SC} d={delay} mode={mode} alpha={alpha} columns={bc}")
    h, J = random_ising(n, n + R, h_max=80, j_max=j_max)
    rng = np.random.default_rng(n)
    q = rng.integers(-6, 7, size=max(SC, 1))[:SC]
    i0 = rng.integers(alpha + 4, 90, size=max(SC, 1))[:SC]
    prob = lib.Problem(h, J)
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=alpha, noise=7, delay=delay, seed=n, mode=mode,
              target=None, block_columns=bc)
    split = run_gpu(prob, split_rows=1, **kw)
    whole = run_gpu(prob, split_rows=-1, **kw)
    _same(split, whole)
    ref = run_oracle(h, J, **{k: v for k, v in kw.items() if k not in ("block_columns",)} | dict(trials=[0, T - 1]))
    assert_same(split, ref, trial_idx=[0, T - 1])
    prob.close()


def test_forced_split_gi_with_target(lib):
    """GI n = 12 (N = 144) at the paper's schedules with target E*: first hits and best energies of the
    split form equal the oracle's for every trial."""
    _note("case split anneal GI n=12 R=16 T=12 SC=120")
    h, J, e_star = gi_case(12, 8)
    q, i0, noise = paper_schedules(120, tau=12)
    prob = lib.Problem(h, J)
    kw = dict(replicas=16, trials=12, cycles=120, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=12,
              target=e_star)
    gpu = run_gpu(prob, split_rows=1, **kw)
    assert_same(gpu, run_oracle(h, J, **kw))
    prob.close()


@pytest.mark.parametrize("n,trials,sampled", [(8, 32, [0, 31]), (20, 8, [0, 7])])
def test_forced_split_ssa_against_oracle(lib, n, trials, sampled):
    """SSA (R = 1, no coupling, Section 4.4 schedule at scale 4) in the split form against the oracle's SSA
    of Eq. 2: energy traces and final counters of sampled trials."""
    _note(f"case split SSA GI n={n} trials={trials}")
    h, J, e_star = gi_case(n, 3, scale=4)
    SC = 300
    i0 = ssqa.scaled(ssqa.ssa_i0_schedule(SC, 10, Fraction(1, 2), 1, 16), 4)
    prob = lib.Problem(h, J)
    gpu = run_gpu(prob, replicas=1, trials=trials, cycles=SC, q=np.zeros(SC, int), i0=i0, alpha=1, noise=4,
                  delay=1, seed=4, target=e_star, split_rows=1)
    e_ref, Is_ref, _ = ssqa.ssa_anneal(h, J, sampled, SC, i0, 1, 4, seed=4, chains=[0])
    assert np.array_equal(gpu["trace"][:, sampled, :], e_ref)
    assert np.array_equal(gpu["Is"][sampled], Is_ref)
    prob.close()


def test_ssa_shape_takes_split_form_by_itself(lib):
    """N = 2500, R = 1, 100 trials (four 32-column blocks, so the automatic choice is the split form): the
    automatic run equals both forced forms bit for bit; trial 0 is replayed by the oracle."""
    _note("case automatic split N=2500 R=1 T=100 SC=30")
    h, J = random_ising(2500, 250, h_max=20, j_max=1, density=0.5)
    rng = np.random.default_rng(250)
    SC = 30
    i0 = rng.integers(4, 64, size=SC)
    prob = lib.Problem(h, J)
    kw = dict(replicas=1, trials=100, cycles=SC, q=np.zeros(SC, int), i0=i0, alpha=1, noise=4, delay=1, seed=9)
    auto = run_gpu(prob, **kw)
    forced = run_gpu(prob, split_rows=1, **kw)
    whole = run_gpu(prob, split_rows=-1, **kw)
    _same(auto, forced)
    _same(auto, whole)
    assert_same(auto, run_oracle(h, J, **(kw | dict(trials=[0]))), trial_idx=[0])
    prob.close()


def test_ssa_table4_shape_long_run_against_oracle(lib):
    """Table 4's SSA at N = 2500 (GI n = 50 at scale 4, R = 1, 100 trials) for its first 1000 cycles of the
    I_0 schedule (Section 4.4): the automatic row-split form with the four waves sharing each tile's K steps
    runs 1000 launches, reusing the ring slots and energy-sum slots hundreds of times; trials 0 and 99 are
    replayed by the oracle's SSA (Eq. 2), energy trace and final counters."""
    _note("case SSA N=2500 T=100 SC=1000 against the oracle")
    h, J, e_star = gi_case(50, 50, scale=4)
    SC = 1000
    i0 = ssqa.scaled(ssqa.ssa_i0_schedule(SC, 10, Fraction(1, 2), 1, 16), 4)
    prob = lib.Problem(h, J)
    assert prob.padded == 2560 and prob.fp4_exact
    gpu = run_gpu(prob, replicas=1, trials=100, cycles=SC, q=np.zeros(SC, int), i0=i0, alpha=1, noise=4,
                  delay=1, seed=50, target=e_star)
    sampled = [0, 99]
    e_ref, Is_ref, _ = ssqa.ssa_anneal(h, J, sampled, SC, i0, 1, 4, seed=50, chains=[0])
    assert np.array_equal(gpu["trace"][:, sampled, :], e_ref)
    assert np.array_equal(gpu["Is"][sampled], Is_ref)
    assert np.array_equal(gpu["best"][sampled], e_ref.min(axis=(0, 2)))
    prob.close()


def test_ssqa_table4_shape_split_against_oracle(lib):
    """Table 4's SSQA at N = 2500 (GI n = 50, R = 25, 100 trials, Table 2 schedules): the automatic choice is the
    row-split form on 50 blocks of 64 columns (groups of four tiles); over its first 200 cycles trials 0 and
    99 equal the oracle (energy trace, best, first hit, final counters), and all trials equal the persistent
    form."""
    _note("case SSQA N=2500 R=25 T=100 SC=200 split against the oracle")
    h, J, e_star = gi_case(50, 50)
    SC = 200
    q, i0, noise = paper_schedules(SC, tau=50)
    prob = lib.Problem(h, J)
    kw = dict(replicas=25, trials=100, cycles=SC, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=50,
              target=e_star)
    auto = run_gpu(prob, **kw)
    whole = run_gpu(prob, split_rows=-1, **kw)
    _same(auto, whole)
    assert_same(auto, run_oracle(h, J, **(kw | dict(trials=[0, 99]))), trial_idx=[0, 99])
    prob.close()
