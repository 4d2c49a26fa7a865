"""GPU tests of the autotuner: every tiling it times runs the anneal bit for bit like the oracle (each is
recorded in the cache in turn and taken by an automatic ssqa_anneal), the chosen one is what later automatic
calls take, the cache survives a save / load, and a tuned batch equals its plain anneals."""

import sys

import numpy as np
import pytest

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
    lib.ssqa_tune_clear()
    yield lib
    lib.ssqa_tune_clear()


def _run(lib, prob, kw):
    import torch
    res = lib.ssqa_anneal(prob, trace=True, final_is=True, **kw)
    torch.cuda.synchronize()
    return {"best": res.best_energy.cpu().numpy(), "first_hit": res.first_hit.cpu().numpy(),
            "trace": res.energy_trace.cpu().numpy(), "Is": res.final_is.cpu().numpy()}


@pytest.mark.parametrize("case", ["gi12_fp4", "ising300_int8_mode1"])
def test_every_candidate_equals_the_oracle(lib, case, tmp_path):
    if case == "gi12_fp4":
        h, J, e_star = gi_case(12, 7)          # N = 144 (2 row tiles, ragged), fp4 and int8 candidates
        q, i0, noise = paper_schedules(50, tau=5)
        kw = dict(replicas=16, trials=40, cycles=50, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=3,
                  target=e_star)
    else:
        h, J = random_ising(300, 5, h_max=80, j_max=9)   # int8 only, general epilogue, both neighbours
        rng = np.random.default_rng(5)
        q = rng.integers(-7, 8, size=40)
        i0 = rng.integers(4, 100, size=40)
        kw = dict(replicas=6, trials=21, cycles=40, jperp=q, i0=i0, alpha=2, noise_amp=9, delay=2, seed=8,
                  coupling_mode=1)
    _note(f"case tune {case}")
    prob = lib.Problem(h, J)
    lib.ssqa_tune_clear()
    tile, tuned = lib.ssqa_tune_lookup(prob, **kw)
    assert not tuned
    chosen, cands = lib.ssqa_tune_anneal(prob, probe_cycles=10, **kw)
    assert len(cands) >= 2 and chosen in cands
    assert all(c["ms_per_cycle"] > 0 for c in cands)
    assert chosen["ms_per_cycle"] == min(c["ms_per_cycle"] for c in cands)
    if case == "gi12_fp4":
        assert {c["operands"] for c in cands} == {"fp4", "int8"}
    else:
        assert {c["operands"] for c in cands} == {"int8"}
    got, tuned = lib.ssqa_tune_lookup(prob, **kw)
    assert tuned and {k: got[k] for k in ("block_columns", "trials_per_block", "operands")} == \
        {k: chosen[k] for k in ("block_columns", "trials_per_block", "operands")}
    # the cache survives a save / clear / load
    path = str(tmp_path / "tune.json")
    lib.ssqa_tune_save(path)
    lib.ssqa_tune_clear()
    assert not lib.ssqa_tune_lookup(prob, **kw)[1]
    assert lib.ssqa_tune_load(path) == 1
    assert lib.ssqa_tune_lookup(prob, **kw)[1]
    # every candidate, recorded in turn, runs an automatic anneal exactly like the oracle
    ref = run_oracle(h, J, replicas=kw["replicas"], trials=kw["trials"], cycles=kw["cycles"], q=q, i0=i0,
                     alpha=kw["alpha"], noise=kw["noise_amp"], delay=kw["delay"], seed=kw["seed"],
                     mode=kw.get("coupling_mode", 0), target=kw.get("target"))
    for c in cands:
        _note(f"  candidate {c['block_columns']} columns x {c['trials_per_block']} trials, {c['operands']}")
        lib.ssqa_tune_set(prob, c, **kw)
        used, tuned = lib.ssqa_tune_lookup(prob, **kw)
        assert tuned and used["block_columns"] == c["block_columns"] and used["operands"] == c["operands"]
        assert used["trials_per_block"] == c["trials_per_block"] and used["blocks"] == c["blocks"]
        assert_same(_run(lib, prob, kw), ref)
    prob.close()


def test_set_refuses_an_illegal_tile(lib):
    _note("case tune set refused")
    h, J = random_ising(100, 9, h_max=50, j_max=7)
    prob = lib.Problem(h, J)
    q = np.zeros(10, dtype=np.int32)
    kw = dict(replicas=40, trials=3, cycles=10, jperp=q, i0=np.full(10, 24), alpha=1, noise_amp=5, delay=1, seed=0)
    with pytest.raises(lib.SSQAError) as err:
        lib.ssqa_tune_set(prob, {"block_columns": 32, "trials_per_block": 1, "operands": "int8"}, **kw)
    assert err.value.name == "SSQA_ENOTSUP"
    with pytest.raises(lib.SSQAError):
        lib.ssqa_tune_anneal(prob, block_columns=64, **kw)
    # 128 columns with int8 operands need J in one int8 plane
    h2, J2 = random_ising(100, 9, h_max=50, j_max=300)
    two = lib.Problem(h2, J2)
    assert two.planes == 2
    kw2 = dict(kw, replicas=8)
    with pytest.raises(lib.SSQAError):
        lib.ssqa_tune_set(two, {"block_columns": 128, "trials_per_block": 1, "operands": "int8"}, **kw2)
    lib.ssqa_tune_set(prob, {"block_columns": 128, "trials_per_block": 1, "operands": "int8"}, **kw2)
    prob.close()
    two.close()


def test_tuned_batch_equals_plain(lib):
    """Twelve uneven GI instances (n from 10 to 40; the larger pad to at least 1024 rows, so 128-column blocks
    are a candidate): the tuned 128-column floor is one of the candidates, a batch created afterwards uses it,
    and every instance's best energy, first hit and energy trace equal its plain anneal."""
    import torch
    _note("case tune batch")
    lib.ssqa_tune_clear()
    pairs = uneven_gi_batch(12, 10, 40, 0.3, 0.7, seed_base=300)
    SC = 60
    jobs = []
    for g, pair in enumerate(pairs):
        h, J, e_star = lib.ssqa_gi_to_ising(pair.a1, pair.a2, 1, 1, 12)
        q, i0, noise = paper_schedules(SC, tau=10)
        jobs.append((lib.Problem(h, J), dict(replicas=32, trials=8, cycles=SC, jperp=q, i0=i0, alpha=1,
                                             noise_amp=noise, delay=1, seed=g, target=e_star)))
    padded = {p.padded for p, _ in jobs}
    assert max(padded) >= 1024
    res = lib.ssqa_tune_batch(jobs, probe_cycles=8)
    assert res["wide_rows"] == 0 or res["wide_rows"] in padded
    assert res["ms_per_cycle"] > 0
    batch = lib.Batch([(p, dict(kw, trace=True)) for p, kw in jobs])
    out = batch.run()
    torch.cuda.synchronize()
    for (p, kw), r in zip(jobs, out):
        ref = lib.ssqa_anneal(p, trace=True, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(r.best_energy.cpu().numpy(), ref.best_energy.cpu().numpy())
        assert np.array_equal(r.first_hit.cpu().numpy(), ref.first_hit.cpu().numpy())
        assert np.array_equal(r.energy_trace.cpu().numpy(), ref.energy_trace.cpu().numpy())
    batch.close()
    for p, _ in jobs:
        p.close()
