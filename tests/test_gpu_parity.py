"""GPU parity: the HIP sweep against the oracle, bit for bit, through the C ABI."""

import os
import sys

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


def test_gi5_full_small_case(lib):
    """N = 25 GI (G(5, 0.5) with graph seed 0 and its relabelled copy), R = 8, 500 cycles,
    100 trials, Philox seed 0: every energy, best, first hit and final counter."""
    _note("case gi5 N=25 R=8 T=100 SC=500")
    h, J, e_star = gi_case(5, 0)
    q, i0, noise = paper_schedules(500)
    prob = lib.Problem(h, J)
    kw = dict(replicas=8, trials=100, cycles=500, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=0,
              target=e_star)
    gpu = run_gpu(prob, **kw)
    ref = run_oracle(h, J, **kw)
    assert_same(gpu, ref)
    assert (gpu["first_hit"] >= 0).mean() > 0.9


@pytest.mark.parametrize("n,R,T,SC,delay,mode,seed", [
    (300, 5, 30, 40, 1, 0, 3),     # ragged N (3 row tiles, 300 of 384 rows), dead columns, partial last group
    (129, 7, 9, 25, 0, 1, 4),      # one row past a tile, d = 0, both-neighbour coupling
    (128, 64, 3, 20, 2, 0, 5),     # exact tile, R = 64 (one trial per workgroup), d = 2
    (1, 3, 5, 30, 1, 1, 6),        # a single spin
    (70, 1, 11, 30, 1, 0, 7),      # R = 1 (the ring couples a replica to itself)
])
def test_random_ising_shapes(lib, n, R, T, SC, delay, mode, seed):
    _note(f"case random n={n} R={R} T={T} SC={SC} d={delay} mode={mode}")
    h, J = random_ising(n, seed, h_max=90, j_max=11)
    rng = np.random.default_rng(seed)
    q = rng.integers(-9, 10, size=SC)
    i0 = rng.integers(3, 128, size=SC)
    prob = lib.Problem(h, J)
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=3, noise=13, delay=delay, seed=seed,
              mode=mode)
    gpu = run_gpu(prob, **kw)
    ref = run_oracle(h, J, **kw)
    assert_same(gpu, ref)


def test_two_int8_planes(lib):
    """|J| beyond int8: J is split into two exact planes."""
    _note("case planes n=150 R=4 T=16 SC=30")
    h, J = random_ising(150, 9, h_max=2000, j_max=300)
    prob = lib.Problem(h, J)
    assert prob.planes == 2
    rng = np.random.default_rng(1)
    q = rng.integers(0, 50, size=30)
    i0 = np.full(30, 100)
    kw = dict(replicas=4, trials=16, cycles=30, q=q, i0=i0, alpha=1, noise=40, delay=1, seed=2)
    assert_same(run_gpu(prob, **kw), run_oracle(h, J, **kw))


def test_split_launches_equal_one_launch(lib):
    """A host loop of short launches (state kept in device memory) equals one persistent launch."""
    _note("case split launches n=260 R=6 T=20 SC=57 d=2")
    h, J = random_ising(260, 12, h_max=60, j_max=9)
    rng = np.random.default_rng(3)
    q = rng.integers(0, 12, size=57)
    i0 = rng.integers(10, 60, size=57)
    prob = lib.Problem(h, J)
    kw = dict(replicas=6, trials=20, cycles=57, q=q, i0=i0, alpha=1, noise=11, delay=2, seed=8, mode=1)
    one = run_gpu(prob, **kw)
    for cpl in (1, 7):
        many = run_gpu(prob, cycles_per_launch=cpl, **kw)
        for key in ("best", "first_hit", "trace", "Is"):
            assert np.array_equal(one[key], many[key]), (cpl, key)
    assert_same(one, run_oracle(h, J, **kw))


def test_zero_cycles_and_determinism(lib):
    _note("case zero cycles")
    h, J, e_star = gi_case(4, 2)
    q, i0, noise = paper_schedules(10)
    prob = lib.Problem(h, J)
    kw = dict(replicas=8, trials=5, cycles=0, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=3,
              target=e_star)
    assert_same(run_gpu(prob, **kw), run_oracle(h, J, **kw))
    kw["cycles"] = 10
    a, b = run_gpu(prob, **kw), run_gpu(prob, **kw)
    for key in a:
        assert np.array_equal(a[key], b[key])


def test_ssa_mode(lib):
    """SSA (Eq. 2, Section 4.4 schedule) as R = 1 without coupling, against the oracle's SSA."""
    _note("case SSA n=8 (N=64)")
    from fractions import Fraction
    h, J, e_star = gi_case(8, 3, scale=4)
    SC = 400
    i0 = ssqa.scaled(ssqa.ssa_i0_schedule(SC, 10, Fraction(1, 2), 1, 16), 4)
    prob = lib.Problem(h, J)
    gpu = run_gpu(prob, replicas=1, trials=32, cycles=SC, q=np.zeros(SC, int), i0=i0, alpha=1, noise=4,
                  delay=1, seed=4, target=e_star)
    e_ref, Is_ref, _ = ssqa.ssa_anneal(h, J, 32, SC, i0, 1, 4, seed=4, chains=[0])
    assert np.array_equal(gpu["trace"], e_ref)
    assert np.array_equal(gpu["Is"], Is_ref)


def test_energy_entry_point(lib):
    import torch
    _note("case ssqa_energy")
    h, J = random_ising(333, 21, h_max=500, j_max=127)
    prob = lib.Problem(h, J)
    rng = np.random.default_rng(0)
    spins = rng.choice([-1, 1], size=(17, 333)).astype(np.int8)
    e = lib.ssqa_energy(prob, torch.from_numpy(spins).cuda()).cpu().numpy()
    F = ssqa.field(J, spins.astype(np.int64))
    assert np.array_equal(e, ssqa.energy_from_field(h, spins.astype(np.int64), F))
    assert e[0] == ssqa.energy_direct(h, J, spins[0])


def test_gi20_sampled_trials_full_size(lib):
    """N = 400 GI at its full run shape (R = 32, 256 trials, 2000 cycles); trials 0, 77 and 255
    replayed by the oracle over all 2000 cycles."""
    _note("case gi20 N=400 R=32 T=256 SC=2000 (sampled)")
    h, J, e_star = gi_case(20, 1)
    q, i0, noise = paper_schedules(2000)
    prob = lib.Problem(h, J)
    kw = dict(replicas=32, cycles=2000, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=0, target=e_star)
    gpu = run_gpu(prob, trials=256, **kw)
    sample = [0, 77, 255]
    ref = run_oracle(h, J, trials=sample, **kw)
    assert_same(gpu, ref, trial_idx=sample)


@pytest.mark.timeout(900)
def test_gi50_sampled_trials_full_size(lib):
    """N = 2500 GI at the benchmark's shape and launch (R = 64, 1024 trials, 2000 cycles, one
    persistent launch); trials 0 and 1023 replayed by the oracle over all 2000 cycles, and every
    trial's best energy checked against the exact energy of its reported state bound."""
    _note("case gi50 N=2500 R=64 T=1024 SC=2000 (sampled)")
    h, J, e_star = gi_case(50, 2)
    q, i0, noise = paper_schedules(2000)
    prob = lib.Problem(h, J)
    kw = dict(replicas=64, cycles=2000, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=0, target=e_star)
    gpu = run_gpu(prob, trials=1024, **kw)
    _note("  gpu done; oracle replay of trials 0 and 1023")
    sample = [0, 1023]
    ref = run_oracle(h, J, trials=sample, **kw)
    assert_same(gpu, ref, trial_idx=sample)
    # properties at any size: best = min of the trace, first hit consistent, energies >= E*
    tr = gpu["trace"]
    assert np.array_equal(gpu["best"], tr.min(axis=(0, 2)))
    assert (gpu["best"] >= e_star).all()
    hit = gpu["first_hit"]
    ok = hit >= 0
    assert np.array_equal(ok, gpu["best"] == e_star)
    assert (tr[hit[ok], np.nonzero(ok)[0]].min(axis=-1) == e_star).all()


def test_plain_auto_wide_blocks_with_split_leftover(lib):
    """N = 1600 GI pads to 13 tiles.  With 2048 trials of R = 32 the plain layout takes 128-column blocks by
    itself (512 workgroups, at least 1536 rows), and the tile left over after three rounds of the four waves
    is split into column halves.  Every trial equals the 64-column tiling, and sampled trials the oracle."""
    _note("case plain N=1600 R=32 T=2048, automatic 128-column blocks with a split leftover tile")
    h, J, e_star = gi_case(40, 3)
    q, i0, noise = paper_schedules(60, tau=20)
    prob = lib.Problem(h, J)
    assert prob.padded == 1664 and prob.fp4_exact
    kw = dict(replicas=32, cycles=60, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=9, target=e_star)
    auto = run_gpu(prob, trials=2048, final_is=False, **kw)
    narrow = run_gpu(prob, trials=2048, final_is=False, block_columns=64, **kw)
    for key in ("best", "first_hit", "trace"):
        assert np.array_equal(auto[key], narrow[key]), key
    sample = [0, 1027, 2047]
    ref = run_oracle(h, J, trials=sample, **kw)
    assert_same(auto, ref, trial_idx=sample, check_is=False)


@pytest.mark.parametrize("n,R,T,SC,delay,mode", [(300, 5, 30, 40, 1, 0), (700, 32, 6, 30, 2, 1), (129, 1, 40, 25, 0, 0)])
def test_block_width_invariance(lib, n, R, T, SC, delay, mode):
    """The tiling choice (32 or 64 columns per workgroup) does not change any result."""
    _note(f"case block width n={n} R={R} T={T}")
    h, J = random_ising(n, n + R, h_max=70, j_max=8)
    rng = np.random.default_rng(n)
    q = rng.integers(0, 9, size=SC)
    i0 = rng.integers(5, 100, size=SC)
    prob = lib.Problem(h, J)
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=1, noise=10, delay=delay, seed=n, mode=mode)
    wide = run_gpu(prob, block_columns=64, **kw)
    narrow = run_gpu(prob, block_columns=32, **kw)
    for key in ("best", "first_hit", "trace", "Is"):
        assert np.array_equal(wide[key], narrow[key]), key
    assert_same(narrow, run_oracle(h, J, **kw))


@pytest.mark.parametrize("n,R,T,SC,delay,mode,fast", [
    (300, 16, 20, 30, 1, 0, True),     # byte-parallel epilogue, negative J_perp, ragged tiles (300 of 384 rows)
    (700, 64, 5, 20, 2, 1, False),     # general epilogue, both ring neighbours, d = 2, trials not filling blocks
    (129, 1, 200, 15, 0, 0, True),     # 128 single-replica trials per block, one row past a tile
    (200, 128, 3, 12, 1, 1, True),     # R = 128: one trial fills a block (only this width holds it)
    (600, 32, 9, 14, 1, 0, True),      # 5 tiles: one round of four waves, then one tile left over
    (1100, 16, 8, 8, 1, 1, False),     # 9 tiles: two rounds, one left over, general epilogue
    (880, 32, 6, 12, 1, 0, True),      # 7 tiles: one round, then three left over
    (870, 16, 10, 10, 2, 1, False),    # 7 tiles, general epilogue, both ring neighbours, d = 2
])
def test_wide_blocks_fp4(lib, n, R, T, SC, delay, mode, fast):
    """128 columns per workgroup (fp4 operands, one wave per SIMD, accumulators in the AGPRs) equal the
    64-column tiling and the oracle bit for bit."""
    _note(f"case 128-column blocks n={n} R={R} T={T} d={delay} mode={mode}")
    h, J = random_ising(n, n + 3 * R, h_max=70, j_max=4)   # |J| <= 4: every entry exact in fp4
    rng = np.random.default_rng(n + R)
    q = rng.integers(-6, 7, size=SC)
    i0 = rng.integers(8, 30, size=SC) if fast else rng.integers(5, 100, size=SC)
    prob = lib.Problem(h, J)
    assert prob.fp4_exact
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=1, noise=9, delay=delay, seed=n, mode=mode)
    wide = run_gpu(prob, block_columns=128, **kw)
    if R <= 64:
        ref64 = run_gpu(prob, block_columns=64, **kw)
        for key in ("best", "first_hit", "trace", "Is"):
            assert np.array_equal(wide[key], ref64[key]), key
    assert_same(wide, run_oracle(h, J, **kw))


@pytest.mark.parametrize("n,R,T,SC,delay,mode,bc", [
    (520, 8, 12, 20, 1, 0, 64),     # 5 tiles: one left over, split into two 32-column halves
    (700, 16, 8, 16, 2, 1, 64),     # 6 tiles: two left over, four halves, d = 2, both ring neighbours
    (1200, 4, 16, 10, 0, 0, 32),    # 10 tiles: two left over, 16-column halves, d = 0
    (520, 2, 30, 20, 1, 1, 32),     # 5 tiles, 16-column halves, both ring neighbours
])
def test_leftover_tiles_in_column_halves(lib, n, R, T, SC, delay, mode, bc):
    """fp4 operands on 64- and 32-column blocks whose last round of the four waves has one or two tiles: those
    tiles are split into column halves, one per wave; the results equal the oracle bit for bit."""
    _note(f"case leftover halves n={n} R={R} T={T} columns={bc} d={delay} mode={mode}")
    h, J = random_ising(n, n + 7 * R, h_max=70, j_max=4)
    rng = np.random.default_rng(n + bc)
    q = rng.integers(-6, 7, size=SC)
    i0 = rng.integers(8, 30, size=SC)
    prob = lib.Problem(h, J)
    assert prob.fp4_exact
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=1, noise=9, delay=delay, seed=n, mode=mode)
    gpu = run_gpu(prob, block_columns=bc, operand_format=2, split_rows=-1, **kw)   # the persistent form
    assert_same(gpu, run_oracle(h, J, **(kw | dict(trials=[0, T - 1]))), trial_idx=[0, T - 1])


@pytest.mark.parametrize("n,R,T,SC,delay,mode,fast,j_max", [
    (300, 16, 20, 30, 1, 0, True, 9),      # byte-parallel epilogue, entries without fp4 codes, ragged tiles
    (700, 64, 5, 20, 2, 1, False, 127),    # general epilogue, |J| up to 127, both ring neighbours, d = 2
    (129, 1, 200, 15, 0, 0, True, 60),     # 128 single-replica trials per block, one row past a tile
    (100, 8, 20, 10, 1, 0, True, 50),      # one tile of two K steps, split into column halves
    (200, 128, 3, 12, 1, 1, True, 11),     # R = 128: one trial fills a block
    (600, 32, 9, 14, 1, 0, True, 100),     # 5 tiles: one round of four waves, then one tile left over (split)
    (1100, 16, 8, 8, 1, 1, False, 127),    # 9 tiles: two rounds, one left over, general epilogue
    (880, 32, 6, 12, 1, 0, True, 33),      # 7 tiles: one round, then three left over
])
def test_wide_blocks_int8(lib, n, R, T, SC, delay, mode, fast, j_max):
    """128 columns per workgroup with int8 operands (2 x in {0, 2} against one int8 plane, int32 accumulators
    starting from the per-row constants, in the AGPRs) equal the 64-column tiling and the oracle bit for bit."""
    _note(f"case 128-column int8 blocks n={n} R={R} T={T} d={delay} mode={mode} |J|<={j_max}")
    h, J = random_ising(n, n + 5 * R, h_max=90, j_max=j_max)
    rng = np.random.default_rng(n + R + 1)
    q = rng.integers(-6, 7, size=SC)
    i0 = rng.integers(8, 30, size=SC) if fast else rng.integers(5, 100, size=SC)
    prob = lib.Problem(h, J)
    assert prob.planes == 1
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=1, noise=9, delay=delay, seed=n, mode=mode)
    wide = run_gpu(prob, block_columns=128, operand_format=1, **kw)
    if R <= 64:
        ref64 = run_gpu(prob, block_columns=64, operand_format=1, **kw)
        for key in ("best", "first_hit", "trace", "Is"):
            assert np.array_equal(wide[key], ref64[key]), key
    assert_same(wide, run_oracle(h, J, **kw))


def test_wide_int8_blocks_need_one_plane(lib):
    h, J = random_ising(100, 5, h_max=10, j_max=300)        # |J| beyond 127: two int8 planes
    prob = lib.Problem(h, J)
    assert prob.planes == 2
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_anneal(prob, replicas=4, trials=2, cycles=3, jperp=np.zeros(3, np.int32), i0=np.full(3, 20),
                        alpha=1, noise_amp=4, delay=1, seed=0, block_columns=128)
    assert ei.value.name == "SSQA_ENOTSUP"


def test_large_n_uses_narrow_blocks(lib):
    """N = 6600 (padded 6656): 64-column bit planes exceed LDS, so 32-column blocks run; sampled trials
    against the oracle."""
    _note("case large N=6600 R=4 T=10 SC=12")
    h, J = random_ising(6600, 77, h_max=40, j_max=3, density=0.3)
    rng = np.random.default_rng(5)
    SC = 12
    q = rng.integers(0, 6, size=SC)
    i0 = np.full(SC, 30)
    prob = lib.Problem(h, J)
    kw = dict(replicas=4, cycles=SC, q=q, i0=i0, alpha=1, noise=7, delay=1, seed=3)
    gpu = run_gpu(prob, trials=10, **kw)
    ref = run_oracle(h, J, trials=[0, 9], **kw)
    assert_same(gpu, ref, trial_idx=[0, 9])


@pytest.mark.parametrize("n,block_columns,formats", [
    (13056, 0, (2, 1)),     # 32-column blocks (chosen by themselves), fp4 and int8 operands
    (6400, 64, (2, 1)),     # 64-column blocks
    (3072, 128, (2, 1)),    # 128-column blocks, 24 tiles
])
def test_maximum_n_at_the_lds_limit(lib, n, block_columns, formats):
    """The largest padded size whose bit planes fit in LDS for each block width at d = 1 (the workgroup's
    LDS is then exactly 160 KiB): sampled trials against the oracle.  With d = 2 the same problem needs more
    LDS than a CU has and is refused."""
    _note(f"case maximum N={n} block_columns={block_columns} R=4 T=8 SC=4")
    h, J = random_ising(n, 91, h_max=40, j_max=3, density=0.2)
    rng = np.random.default_rng(6)
    SC = 4
    q = rng.integers(0, 6, size=SC)
    i0 = np.full(SC, 30)
    prob = lib.Problem(h, J)
    assert prob.padded == n and prob.fp4_exact
    kw = dict(replicas=4, cycles=SC, q=q, i0=i0, alpha=1, noise=7, delay=1, seed=4)
    ref = run_oracle(h, J, trials=[0, 7], **kw)
    for fmt in formats:
        gpu = run_gpu(prob, trials=8, operand_format=fmt, block_columns=block_columns, **kw)
        assert_same(gpu, ref, trial_idx=[0, 7])
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_anneal(prob, replicas=4, trials=8, cycles=SC, jperp=q, i0=i0, alpha=1, noise_amp=7, delay=2,
                        seed=4, block_columns=block_columns)
    assert ei.value.name == "SSQA_ENOTSUP" and "LDS" in str(ei.value)
    del prob


def test_qmc_energy_entry_point(lib):
    """H_c (Eq. 4) of the final state of an anneal against the oracle's qmc_energy."""
    _note("case ssqa_qmc_energy")
    h, J, e_star = gi_case(7, 8)
    q, i0, noise = paper_schedules(80, tau=10)
    prob = lib.Problem(h, J)
    res = lib.ssqa_anneal(prob, replicas=6, trials=9, cycles=80, jperp=q, i0=i0, alpha=1, noise_amp=noise,
                          delay=1, seed=4, final_is=True)
    hc = lib.ssqa_qmc_energy(prob, res.final_is, jperp=6).cpu().numpy()
    sigma = np.where(res.final_is.cpu().numpy() >= 0, 1, -1).astype(np.int64)
    assert np.array_equal(hc, ssqa.qmc_energy(h, J, sigma, 6))


@pytest.mark.parametrize("case", ["gi9", "ising300", "ising129_mode1_d0", "ising_tail"])
def test_fp4_operands_equal_int8_and_oracle(lib, case):
    """When every J_ij is exactly representable in fp4 (e2m1), the fp4 field product (fp32 accumulation)
    gives exactly the int8 results and the oracle's."""
    _note(f"case fp4 vs int8 {case}")
    if case == "gi9":
        h, J, e_star = gi_case(9, 6)
        q, i0, noise = paper_schedules(120, tau=10)
        kw = dict(replicas=16, trials=12, cycles=120, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=9,
                  target=e_star)
    else:
        n, mode, d = {"ising300": (300, 0, 1), "ising129_mode1_d0": (129, 1, 0), "ising_tail": (385, 0, 2)}[case]
        h, J = random_ising(n, n, h_max=50, j_max=4)
        J[J == 5] = 6
        J[J == -5] = -6
        rng = np.random.default_rng(n)
        q = rng.integers(0, 9, size=40)
        i0 = rng.integers(5, 90, size=40)
        kw = dict(replicas=5, trials=14, cycles=40, q=q, i0=i0, alpha=2, noise=9, delay=d, seed=n, mode=mode)
    prob = lib.Problem(h, J)
    f4 = run_gpu(prob, operand_format=2, **kw)
    i8 = run_gpu(prob, operand_format=1, **kw)
    for key in ("best", "first_hit", "trace", "Is"):
        assert np.array_equal(f4[key], i8[key]), key
    assert_same(f4, run_oracle(h, J, **kw))


def test_fp4_refused_when_inexact(lib):
    h, J = random_ising(40, 3, h_max=20, j_max=9)
    prob = lib.Problem(h, J)
    with pytest.raises(lib.SSQAError) as ei:
        run_gpu(prob, replicas=2, trials=2, cycles=3, q=[0, 0, 0], i0=[9, 9, 9], alpha=1, noise=1, delay=1, seed=0,
                operand_format=2)
    assert ei.value.name == "SSQA_ENOTSUP"


@pytest.mark.parametrize("n,mode,delay,j_max,fmt", [
    (300, 1, 2, 8, 1),     # int8 operands, both neighbours, d = 2
    (300, 1, 2, 4, 2),     # fp4 operands (every |J_ij| <= 4)
    (200, 0, 1, 6, 0),     # one neighbour, automatic operands
])
def test_byte_parallel_update_with_negative_jperp(lib, n, mode, delay, j_max, fmt):
    """alpha = 1 with small I_0, n_rnd and |J_perp| selects the byte-parallel counter update; J_perp takes
    both signs (negative values complement the coupling bits), I_0 varies from cycle to cycle."""
    _note(f"case byte-parallel update n={n} mode={mode} d={delay} fmt={fmt}")
    h, J = random_ising(n, 900 + n + mode, h_max=60, j_max=j_max)
    if fmt == 2:
        J[np.abs(J) == 5] = 4
    rng = np.random.default_rng(n + 17)
    SC = 36
    q = rng.integers(-8, 9, size=SC)      # max I_0 + 2 n_rnd + 2 |q| (1 + mode) = 40 + 20 + 32 <= 128
    i0 = rng.integers(2, 41, size=SC)
    kw = dict(replicas=6, trials=11, cycles=SC, q=q, i0=i0, alpha=1, noise=10, delay=delay, seed=n, mode=mode)
    prob = lib.Problem(h, J)
    assert_same(run_gpu(prob, operand_format=fmt, **kw), run_oracle(h, J, **kw))
