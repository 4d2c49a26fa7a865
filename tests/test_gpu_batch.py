"""GPU tests of the batched form: many anneals of uneven size in one persistent launch replayed from
a HIP graph give, anneal by anneal, exactly the results of separate ssqa_anneal calls and of the oracle."""

import sys

import numpy as np
import pytest

from oracle import gi
from synth import random_ising, uneven_gi_batch
from tests.parity_util import assert_same, gi_case, paper_schedules, run_oracle

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


def _host(res):
    return {
        "best": res.best_energy.cpu().numpy(),
        "first_hit": res.first_hit.cpu().numpy(),
        "trace": res.energy_trace.cpu().numpy() if res.energy_trace is not None else None,
        "Is": res.final_is.cpu().numpy() if res.final_is is not None else None,
    }


def _mixed_jobs(lib):
    rng = np.random.default_rng(11)
    jobs = []
    specs = [
        # (kind, size, R, T, SC, delay, mode, alpha)
        ("gi", 5, 8, 40, 60, 1, 0, 1),
        ("ising", 300, 5, 13, 45, 1, 0, 1),
        ("ising", 129, 7, 9, 30, 0, 1, 1),
        ("gi", 12, 32, 70, 50, 2, 0, 1),
        ("ising", 200, 4, 20, 25, 1, 0, 3),
        ("ising", 64, 64, 3, 40, 1, 1, 2),
    ]
    models = []
    for idx, (kind, size, R, T, SC, d, mode, alpha) in enumerate(specs):
        if kind == "gi":
            h, J, e_star = gi_case(size, idx)
            q, i0, noise = paper_schedules(SC, tau=10)
        else:
            h, J = random_ising(size, 40 + idx, h_max=80, j_max=9)
            e_star = None
            q = rng.integers(0, 12, size=SC)
            i0 = rng.integers(alpha, 90, size=SC)
            noise = 9
        prob = lib.Problem(h, J)
        kw = dict(replicas=R, trials=T, cycles=SC, jperp=q, i0=i0, alpha=alpha, noise_amp=noise, delay=d,
                  seed=100 + idx, coupling_mode=mode, target=e_star)
        jobs.append((prob, kw))
        models.append((h, J))
    return jobs, models


def test_batch_equals_separate_anneals_and_oracle(lib):
    import torch
    _note("case mixed batch of 6 anneals (3 kernel variants)")
    jobs, models = _mixed_jobs(lib)
    batch = lib.Batch([(p, dict(kw, trace=True, final_is=True)) for p, kw in jobs])
    assert batch.blocks > 0
    results = [_host(r) for r in batch.run()]
    torch.cuda.synchronize()
    for i, (prob, kw) in enumerate(jobs):
        alone = lib.ssqa_anneal(prob, trace=True, final_is=True, **kw)
        torch.cuda.synchronize()
        a = _host(alone)
        for key in ("best", "first_hit", "trace", "Is"):
            assert np.array_equal(results[i][key], a[key]), (i, key)
    # the oracle on every anneal
    for i, ((prob, kw), (h, J)) in enumerate(zip(jobs, models)):
        ref = run_oracle(h, J, replicas=kw["replicas"], trials=kw["trials"], cycles=kw["cycles"], q=kw["jperp"],
                         i0=kw["i0"], alpha=kw["alpha"], noise=kw["noise_amp"], delay=kw["delay"], seed=kw["seed"],
                         mode=kw["coupling_mode"], target=kw["target"])
        assert_same(results[i], ref)
    # graph replays, with eager work in between, reproduce the first run
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()
        again = [_host(r) for r in batch.run()]
        torch.cuda.synchronize()
        float(junk)
        for i in range(len(jobs)):
            for key in ("best", "first_hit", "trace", "Is"):
                assert np.array_equal(again[i][key], results[i][key]), (rep, i, key)
    batch.close()


def test_batch_with_wide_blocks(lib):
    """Anneals asking for 128 columns per workgroup (fp4 operands, both epilogues, both coupling modes) in one
    batch with a 64-column int8 anneal: each equals its separate anneal and the oracle."""
    import torch
    _note("case batch with 128-column blocks")
    rng = np.random.default_rng(12)
    jobs, models = [], []
    h, J, e_star = gi_case(6, 21)
    q, i0, noise = paper_schedules(40, tau=10)
    jobs.append((lib.Problem(h, J), dict(replicas=16, trials=20, cycles=40, jperp=q, i0=i0, alpha=1,
                                         noise_amp=noise, delay=1, seed=7, coupling_mode=0, target=e_star,
                                         block_columns=128)))
    models.append((h, J))
    h, J = random_ising(150, 9, h_max=60, j_max=4)
    jobs.append((lib.Problem(h, J), dict(replicas=32, trials=7, cycles=30, jperp=rng.integers(-5, 6, size=30),
                                         i0=rng.integers(2, 90, size=30), alpha=2, noise_amp=8, delay=2, seed=8,
                                         coupling_mode=1, target=None, block_columns=128)))
    models.append((h, J))
    h, J = random_ising(90, 10, h_max=60, j_max=9)       # int8 operands, 64 columns
    jobs.append((lib.Problem(h, J), dict(replicas=8, trials=11, cycles=25, jperp=rng.integers(0, 6, size=25),
                                         i0=rng.integers(1, 60, size=25), alpha=1, noise_amp=6, delay=0, seed=9,
                                         coupling_mode=0, target=None)))
    models.append((h, J))
    batch = lib.Batch([(p, dict(kw, trace=True, final_is=True)) for p, kw in jobs])
    results = [_host(r) for r in batch.run()]
    torch.cuda.synchronize()
    for i, ((prob, kw), (h, J)) in enumerate(zip(jobs, models)):
        alone = _host(lib.ssqa_anneal(prob, trace=True, final_is=True, **kw))
        torch.cuda.synchronize()
        for key in ("best", "first_hit", "trace", "Is"):
            assert np.array_equal(results[i][key], alone[key]), (i, key)
        ref = run_oracle(h, J, replicas=kw["replicas"], trials=kw["trials"], cycles=kw["cycles"], q=kw["jperp"],
                         i0=kw["i0"], alpha=kw["alpha"], noise=kw["noise_amp"], delay=kw["delay"], seed=kw["seed"],
                         mode=kw["coupling_mode"], target=kw["target"])
        assert_same(results[i], ref)
    batch.close()


def test_batch_widens_blocks_from_1024_rows(lib):
    """The batch picks 128-column blocks by itself for an fp4 anneal of at least 1024 padded rows (R = 16,
    T = 24: three workgroups of eight trials), and keeps 64 columns below that (N = 841 pads to 896: six
    workgroups of four trials).  N = 1089 pads to 9 tiles, so the tile left over after two rounds of the four
    waves is split into column halves.  Each anneal still equals its separate anneal and the oracle."""
    import torch
    _note("case batch choosing 128-column blocks at N = 1024 and 1089")
    jobs, models = [], []
    for n, seed in ((32, 31), (29, 32), (33, 33)):
        h, J, e_star = gi_case(n, seed)
        q, i0, noise = paper_schedules(40, tau=10)
        prob = lib.Problem(h, J)
        assert prob.fp4_exact
        jobs.append((prob, dict(replicas=16, trials=24, cycles=40, jperp=q, i0=i0, alpha=1, noise_amp=noise,
                                delay=1, seed=13 + n, coupling_mode=0, target=e_star)))
        models.append((h, J))
    assert [p.padded for p, _ in jobs] == [1024, 896, 1152]
    alone_blocks = [lib.Batch([j]) for j in jobs]
    assert [b.blocks for b in alone_blocks] == [3, 6, 3]
    for b in alone_blocks:
        b.close()
    batch = lib.Batch([(p, dict(kw, trace=True, final_is=True)) for p, kw in jobs])
    assert batch.blocks == 12
    results = [_host(r) for r in batch.run()]
    torch.cuda.synchronize()
    for i, ((prob, kw), (h, J)) in enumerate(zip(jobs, models)):
        alone = _host(lib.ssqa_anneal(prob, trace=True, final_is=True, **kw))
        torch.cuda.synchronize()
        for key in ("best", "first_hit", "trace", "Is"):
            assert np.array_equal(results[i][key], alone[key]), (i, key)
        ref = run_oracle(h, J, replicas=kw["replicas"], trials=kw["trials"], cycles=kw["cycles"], q=kw["jperp"],
                         i0=kw["i0"], alpha=kw["alpha"], noise=kw["noise_amp"], delay=kw["delay"], seed=kw["seed"],
                         mode=kw["coupling_mode"], target=kw["target"])
        assert_same(results[i], ref)
    batch.close()


def test_uneven_gi_batch(lib):
    """Forty GI instances of uneven size (n from 10 to 50, edge probability 0.3-0.7), R = 32, T = 64, in
    one launch: every instance equals its separate anneal; the two smallest instances are replayed by the
    oracle on two trials, and the largest on two trials with its energy trace and final counters."""
    import torch
    _note("case uneven GI batch of 40")
    pairs = uneven_gi_batch(40, seed_base=1000)
    SC = 120
    q, i0, noise = paper_schedules(SC, tau=10)
    jobs, models = [], []
    for g, pair in enumerate(pairs):
        h, J, e_star = lib.ssqa_gi_to_ising(pair.a1, pair.a2, 1, 1, 12)
        prob = lib.Problem(h, J)
        jobs.append((prob, dict(replicas=32, trials=64, cycles=SC, jperp=q, i0=i0, alpha=1, noise_amp=noise,
                                delay=1, seed=g, target=e_star)))
        models.append((h, J, e_star))
    largest = max(range(len(pairs)), key=lambda g: pairs[g].n)
    jobs[largest][1].update(trace=True, final_is=True)
    batch = lib.Batch(jobs)
    res = [_host(r) for r in batch.run()]
    torch.cuda.synchronize()
    for i, (prob, kw) in enumerate(jobs):
        a = _host(lib.ssqa_anneal(prob, **kw))
        torch.cuda.synchronize()
        assert np.array_equal(res[i]["best"], a["best"]) and np.array_equal(res[i]["first_hit"], a["first_hit"]), i
    small = sorted(range(len(pairs)), key=lambda g: pairs[g].n)[:2]
    for g in small:
        h, J, e_star = models[g]
        kw = jobs[g][1]
        ref = run_oracle(h, J, replicas=32, trials=[0, 63], cycles=SC, q=q, i0=i0, alpha=1, noise=noise, delay=1,
                         seed=g, target=e_star)
        assert np.array_equal(res[g]["best"][[0, 63]], ref.best)
        assert np.array_equal(res[g]["first_hit"][[0, 63]], ref.first_hit)
        assert (res[g]["best"] >= e_star).all()
    h, J, e_star = models[largest]
    _note(f"case uneven GI batch: oracle replay of the largest instance, N = {len(h)}")
    ref = run_oracle(h, J, replicas=32, trials=[0, 63], cycles=SC, q=q, i0=i0, alpha=1, noise=noise, delay=1,
                     seed=largest, target=e_star)
    assert_same(res[largest], ref, trial_idx=[0, 63])
    batch.close()
