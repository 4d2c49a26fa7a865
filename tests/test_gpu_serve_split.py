"""GPU tests of the served row-split form: a request whose rows are spread over row groups of workgroups (one
launch per cycle, sigma exchanged through device memory) gives, trial for trial, the best energies and first
hits of ssqa_anneal, alone and beside requests of the persistent form, across step boundaries, for both operand
types, delays 0 to 2, both coupling modes and the general epilogue; a sampled trial is replayed by the oracle."""

import sys

import numpy as np
import pytest

from synth import random_gi_pair, random_ising
from tests.parity_util import paper_schedules

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


def _drain(server, ids, max_steps=10000):
    for _ in range(max_steps):
        server.step()
        if all(server.poll(i)["state"] in ("done", "failed", "cancelled") for i in ids):
            return
    raise AssertionError("requests did not finish")


def _compare(lib, h, J, kw, info):
    import torch
    prob = lib.Problem(h, J)
    ref = lib.ssqa_anneal(prob, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(info["best"], ref.best_energy.cpu().numpy())
    assert np.array_equal(info["first_hit"], ref.first_hit.cpu().numpy())
    prob.close()


@pytest.mark.parametrize("n,R,T,SC,K,delay,mode,alpha,j_max,fp4", [
    (1000, 32, 6, 37, 10, 1, 0, 1, 4, True),      # fp4, 8 tiles in 2 row groups of 4, K not dividing SC
    (900, 8, 13, 25, 7, 2, 1, 3, 60, False),      # int8, d = 2, both neighbours, general epilogue, 64 columns
    (1300, 5, 9, 20, 20, 0, 0, 1, 11, False),     # d = 0, 11 tiles (last group of 3), one step
    (600, 16, 40, 31, 4, 1, 1, 2, 4, True),       # fp4, 5 tiles, many column blocks, alpha = 2
])
def test_split_request_equals_anneal(lib, n, R, T, SC, K, delay, mode, alpha, j_max, fp4):
    _note(f"case split request n={n} R={R} T={T} SC={SC} K={K} d={delay} mode={mode} alpha={alpha} fp4={fp4}")
    h, J = random_ising(n, n + R, h_max=80, j_max=j_max)
    rng = np.random.default_rng(n)
    q = rng.integers(-6, 7, size=SC)
    i0 = rng.integers(alpha + 4, 90, size=SC)
    kw = dict(replicas=R, trials=T, cycles=SC, jperp=q, i0=i0, alpha=alpha, noise_amp=7, delay=delay, seed=n,
              coupling_mode=mode, target=-10 ** 9)
    s = lib.Server(cycles_per_step=K, split_rows=512)
    r = s.submit(h, J, **kw)
    _drain(s, [r])
    x = s.poll(r)
    assert x["state"] == "done" and x["cycles_done"] == SC
    if fp4:
        assert lib.Problem(h, J).fp4_exact
    _compare(lib, h, J, kw, x)
    s.close()


def test_split_beside_persistent_requests_with_early_exit(lib):
    """A forced-split GI request (n = 34, N = 1156, 10 tiles) beside two small requests of the persistent form,
    all with early exit at E*: every request's per-trial results equal ssqa_anneal's up to its retiring step
    (trials that reached E* by then hold E*); the split request's trial 3 is replayed by the oracle."""
    import torch
    from oracle import gi, ssqa
    _note("case split beside persistent requests, early exit")
    SC, K = 60, 12
    q, i0, noise = paper_schedules(SC, tau=6)
    reqs = []
    for n, seed in ((34, 71), (6, 72), (9, 73)):
        pair = random_gi_pair(n, 0.5, 900 + seed)
        h, J, e_star = lib.ssqa_gi_to_ising(pair.a1, pair.a2, 1, 1, 12)
        kw = dict(replicas=32, trials=8, cycles=SC, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=seed,
                  target=e_star)
        reqs.append((pair, h, J, e_star, kw))
    s = lib.Server(cycles_per_step=K, split_rows=1024)
    ids = [s.submit(h, J, early_exit=True, **kw) for _, h, J, _, kw in reqs]
    _drain(s, ids)
    for rid, (pair, h, J, e_star, kw) in zip(ids, reqs):
        x = s.poll(rid)
        assert x["state"] == "done"
        prob = lib.Problem(h, J)
        ref = lib.ssqa_anneal(prob, **dict(kw, cycles=SC))
        torch.cuda.synchronize()
        rb, rh = ref.best_energy.cpu().numpy(), ref.first_hit.cpu().numpy()
        done = x["cycles_done"]
        # energies of cycles 0 .. done - 1 were evaluated (and of cycle SC after the last step)
        limit = SC + 1 if done == SC else done
        hit = (rh >= 0) & (rh < limit)
        assert np.array_equal(x["first_hit"][hit], rh[hit])
        assert (x["first_hit"][~hit] == -1).all()
        assert (x["best"][hit] == e_star).all()
        if done == SC:
            assert np.array_equal(x["best"], rb)
        prob.close()
    pair, h, J, e_star, kw = reqs[0]
    x = s.poll(ids[0])
    done = x["cycles_done"]
    ho, Jo, eo = gi.gi_ising(pair.a1, pair.a2, 12)
    assert eo == e_star
    orc = ssqa.anneal(ho, Jo, 32, [3], SC, q, i0, 1, noise, 1, seed=71, target=e_star)
    limit = SC + 1 if done == SC else done
    expect = orc.first_hit[0] if 0 <= orc.first_hit[0] < limit else -1
    assert x["first_hit"][3] == expect
    s.close()


def test_several_split_requests_at_once(lib):
    """Five forced-split requests of different sizes in flight together (spread over the server's side streams,
    two sharing one) beside a persistent one: each equals ssqa_anneal trial for trial."""
    _note("case several split requests at once")
    s = lib.Server(cycles_per_step=9, split_rows=512)
    jobs = []
    for k, (n, R, T, SC) in enumerate(((700, 8, 10, 30), (520, 16, 6, 25), (1000, 4, 9, 40), (650, 32, 3, 33),
                                       (800, 8, 8, 20), (90, 8, 5, 30))):
        h, J = random_ising(n, 300 + k, h_max=60, j_max=4 if k % 2 else 30)
        rng = np.random.default_rng(300 + k)
        q = rng.integers(-5, 6, size=SC)
        i0 = rng.integers(6, 60, size=SC)
        kw = dict(replicas=R, trials=T, cycles=SC, jperp=q, i0=i0, alpha=1, noise_amp=6, delay=1 + k % 2, seed=k,
                  coupling_mode=k % 2, target=-10 ** 9)
        jobs.append((h, J, kw, s.submit(h, J, **kw)))
    _drain(s, [rid for *_, rid in jobs])
    for h, J, kw, rid in jobs:
        x = s.poll(rid)
        assert x["state"] == "done" and x["cycles_done"] == kw["cycles"]
        _compare(lib, h, J, kw, x)
    s.close()
