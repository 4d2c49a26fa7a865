"""GPU tests of the request server: continuous batching gives every request the result it gets alone
(and that ssqa_anneal gives), admission follows the memory budget, early exit and cancellation work."""

import sys

import numpy as np
import pytest

from synth import random_gi_pair
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


def _request(lib, n, seed, SC=300, R=32, T=16, tau=10):
    pair = random_gi_pair(n, 0.5, 500 + seed)
    h, J, e_star = lib.ssqa_gi_to_ising(pair.a1, pair.a2, 1, 1, 12)
    q, i0, noise = paper_schedules(SC, tau=tau)
    kw = dict(replicas=R, trials=T, cycles=SC, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=seed,
              target=e_star)
    return h, J, kw


def _drain(server, ids, max_steps=10000):
    for _ in range(max_steps):
        server.step()
        if all(server.poll(i)["state"] in ("done", "failed", "cancelled") for i in ids):
            return
    raise AssertionError("requests did not finish")


def test_alone_equals_in_mix_and_equals_anneal(lib):
    """Request A gives the same per-trial best energies and first hits alone, in a mix with requests
    of other sizes arriving at other steps, and from ssqa_anneal (no early exit)."""
    import torch
    _note("case serve alone == mix")
    hA, JA, kwA = _request(lib, 9, 1, SC=300)
    alone = lib.Server(cycles_per_step=40)
    a = alone.submit(hA, JA, **kwA)
    _drain(alone, [a])
    ra = alone.poll(a)
    assert ra["state"] == "done" and ra["cycles_done"] == 300
    ref = lib.ssqa_anneal(lib.Problem(hA, JA), **kwA)
    torch.cuda.synchronize()
    assert np.array_equal(ra["best"], ref.best_energy.cpu().numpy())
    assert np.array_equal(ra["first_hit"], ref.first_hit.cpu().numpy())

    mix = lib.Server(cycles_per_step=40)
    others = [mix.submit(*_request(lib, n, 10 + n, SC=200)[:2], **_request(lib, n, 10 + n, SC=200)[2])
              for n in (5, 20)]
    mix.step()
    a2 = mix.submit(hA, JA, **kwA)
    mix.step()
    others.append(mix.submit(*_request(lib, 14, 3, SC=500)[:2], **_request(lib, 14, 3, SC=500)[2]))
    _drain(mix, others + [a2])
    rb = mix.poll(a2)
    assert np.array_equal(ra["best"], rb["best"]) and np.array_equal(ra["first_hit"], rb["first_hit"])
    alone.close()
    mix.close()


def test_early_exit_is_deterministic(lib):
    """With early exit a request retires at the first step boundary where some trial reached E*; the
    result is the same alone and in a mix, and the trials that hit agree with the full anneal."""
    _note("case serve early exit")
    h, J, kw = _request(lib, 6, 4, SC=600)
    s1 = lib.Server(cycles_per_step=25)
    r1 = s1.submit(h, J, early_exit=True, **kw)
    _drain(s1, [r1])
    x = s1.poll(r1)
    assert x["state"] == "done" and x["cycles_done"] % 25 == 0 and x["cycles_done"] < 600
    assert (x["best"] == kw["target"]).any()
    s2 = lib.Server(cycles_per_step=25, max_active=3)
    ids = [s2.submit(*_request(lib, 12, 7, SC=300)[:2], **_request(lib, 12, 7, SC=300)[2])]
    r2 = s2.submit(h, J, early_exit=True, **kw)
    _drain(s2, ids + [r2])
    y = s2.poll(r2)
    assert y["cycles_done"] == x["cycles_done"]
    assert np.array_equal(x["best"], y["best"]) and np.array_equal(x["first_hit"], y["first_hit"])
    full = lib.ssqa_anneal(lib.Problem(h, J), **kw)
    fh = full.first_hit.cpu().numpy()
    hit = x["first_hit"] >= 0
    assert np.array_equal(x["first_hit"][hit], fh[hit])
    s1.close()
    s2.close()


def test_memory_admission_and_refusal(lib):
    """A budget that holds one n = 12 request runs such requests one at a time; a request larger than
    the whole budget is refused with SSQA_ENOMEM while the others complete."""
    _note("case serve admission")
    reqs = [_request(lib, 12, 20 + k, SC=100) for k in range(3)]
    probe = lib.Server(cycles_per_step=50)
    pid = probe.submit(reqs[0][0], reqs[0][1], **reqs[0][2])
    probe.step()
    one = probe.poll(pid)["memory_bytes"]
    probe.close()
    s = lib.Server(cycles_per_step=50, memory_budget=int(one * 1.5))
    ids = [s.submit(h, J, **kw) for h, J, kw in reqs]
    big_h, big_J, big_kw = _request(lib, 40, 30, SC=100)
    big = s.submit(big_h, big_J, **big_kw)
    max_active = 0
    for _ in range(100):
        s.step()
        st = s.stats()
        max_active = max(max_active, st["active"])
        assert st["memory_in_use"] <= int(one * 1.5)
        if all(s.poll(i)["state"] in ("done", "failed") for i in ids + [big]):
            break
    assert max_active == 1
    assert all(s.poll(i)["state"] == "done" for i in ids)
    fb = s.poll(big)
    assert fb["state"] == "failed" and fb["status"] == -2
    s.close()


def test_cancel(lib):
    _note("case serve cancel")
    s = lib.Server(cycles_per_step=20)
    h, J, kw = _request(lib, 10, 40, SC=400)
    keep = s.submit(h, J, **kw)
    drop = s.submit(*_request(lib, 11, 41, SC=400)[:2], **_request(lib, 11, 41, SC=400)[2])
    s.step()
    s.cancel(drop)
    _drain(s, [keep, drop])
    assert s.poll(drop)["state"] == "cancelled"
    assert s.poll(keep)["state"] == "done" and s.poll(keep)["cycles_done"] == 400
    assert s.stats()["memory_in_use"] == 0
    s.close()


def test_r64_request_equals_anneal(lib):
    """A request with R = 64 replicas (one trial per 64-column block) is admitted, charged and run like any
    other, alone and beside an R = 32 request, and equals ssqa_anneal."""
    import torch
    _note("case serve R=64")
    h, J, kw = _request(lib, 8, 50, SC=120, R=64, T=5)
    s = lib.Server(cycles_per_step=40)
    other = s.submit(*_request(lib, 7, 51, SC=80)[:2], **_request(lib, 7, 51, SC=80)[2])
    r = s.submit(h, J, **kw)
    _drain(s, [other, r])
    x = s.poll(r)
    assert x["state"] == "done" and x["cycles_done"] == 120 and x["memory_bytes"] > 0
    ref = lib.ssqa_anneal(lib.Problem(h, J), **kw)
    torch.cuda.synchronize()
    assert np.array_equal(x["best"], ref.best_energy.cpu().numpy())
    assert np.array_equal(x["first_hit"], ref.first_hit.cpu().numpy())
    s.close()


def test_large_request_in_a_mix(lib):
    """An N = 10^4 GI request (n = 100; J of 100 MB as int32) served beside two small ones gives, trial for
    trial, the best energy and first hit of ssqa_anneal; trial 5 is replayed by the oracle over all cycles."""
    import torch
    from oracle import gi, ssqa
    from tests.parity_util import paper_schedules as sched
    _note("case serve N=10^4 in a mix")
    SC, R, T = 40, 32, 16
    pair = random_gi_pair(100, 0.5, 5003)
    h, J, e_star = lib.ssqa_gi_to_ising(pair.a1, pair.a2, 1, 1, 12)
    q, i0, noise = sched(SC, tau=10)
    kw = dict(replicas=R, trials=T, cycles=SC, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=77,
              target=e_star)
    s = lib.Server(cycles_per_step=15)
    small = [s.submit(*_request(lib, n, 60 + n, SC=60)[:2], **_request(lib, n, 60 + n, SC=60)[2]) for n in (6, 12)]
    big = s.submit(h, J, **kw)
    _drain(s, small + [big])
    x = s.poll(big)
    assert x["state"] == "done" and x["cycles_done"] == SC
    prob = lib.Problem(h, J)
    ref = lib.ssqa_anneal(prob, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(x["best"], ref.best_energy.cpu().numpy())
    assert np.array_equal(x["first_hit"], ref.first_hit.cpu().numpy())
    prob.close()
    del ref
    ho, Jo, eo = gi.gi_ising(pair.a1, pair.a2, 12)
    assert eo == e_star
    orc = ssqa.anneal(ho, Jo, R, [5], SC, q, i0, 1, noise, 1, seed=77, target=e_star)
    assert x["best"][5] == orc.best[0] and x["first_hit"][5] == orc.first_hit[0]
    s.close()
