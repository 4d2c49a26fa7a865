"""GPU tests of ssqa_anneal_noalloc (the anneal whose device state lives in the library's fixed per-device
scratch) against ssqa_anneal, through the C ABI: two calls in a row, the second smaller, each equal bit for
bit to ssqa_anneal on the same inputs; a checkpoint / resume through it; and the refusal of an anneal whose
state exceeds the scratch."""

import sys

import numpy as np
import pytest

from synth import random_ising
from tests.parity_util import gi_case, paper_schedules, run_oracle

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


def _both(lib, prob, **kw):
    """The same anneal through ssqa_anneal_noalloc and ssqa_anneal (in that order), results on the host."""
    import torch
    a = lib.ssqa_anneal_noalloc(prob, **kw)
    torch.cuda.synchronize()
    got = _host(a)
    b = lib.ssqa_anneal(prob, **kw)
    torch.cuda.synchronize()
    return got, _host(b)


def _equal(x, y):
    for key in ("best", "first_hit", "trace", "Is"):
        if x[key] is None:
            assert y[key] is None
            continue
        assert x[key].shape == y[key].shape, key
        if not np.array_equal(x[key], y[key]):
            bad = np.argwhere(x[key] != y[key])
            raise AssertionError(f"{key} differs at {len(bad)} entries, first {bad[0].tolist()}")


def test_two_calls_second_smaller(lib):
    """Call 1: GI n = 30 (N = 900, 1024 padded rows), R = 64, T = 512 (about 36 MiB of counters and history,
    most of the scratch).  Call 2: a ragged random model, N = 90, R = 5, T = 7, d = 2, both-neighbour coupling,
    alpha = 3, on the same scratch that call 1 left full.  Each equals ssqa_anneal bit for bit (trace, best,
    first hit, final counters); call 2 also equals the oracle."""
    h, J, e_star = gi_case(30, 4)
    q, i0, noise = paper_schedules(60, tau=10)
    prob = lib.Problem(h, J)
    kw = dict(replicas=64, trials=512, cycles=60, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=11,
              target=e_star, trace=True, final_is=True)
    _note("case noalloc call 1: GI N=900 R=64 T=512 SC=60")
    got, ref = _both(lib, prob, **kw)
    _equal(got, ref)
    prob.close()

    _note("case noalloc call 2: random N=90 R=5 T=7 SC=50 d=2 mode=1")
    h2, J2 = random_ising(90, 3, h_max=70, j_max=9)
    rng = np.random.default_rng(3)
    q2 = rng.integers(-8, 9, size=50)
    i02 = rng.integers(4, 128, size=50)
    prob2 = lib.Problem(h2, J2)
    kw2 = dict(replicas=5, trials=7, cycles=50, jperp=q2, i0=i02, alpha=3, noise_amp=11, delay=2, seed=5,
               coupling_mode=1, trace=True, final_is=True)
    got2, ref2 = _both(lib, prob2, **kw2)
    _equal(got2, ref2)
    orc = run_oracle(h2, J2, replicas=5, trials=7, cycles=50, q=q2, i0=i02, alpha=3, noise=11, delay=2, seed=5,
                     mode=1)
    assert np.array_equal(got2["trace"], orc.energy)
    assert np.array_equal(got2["Is"], orc.Is)
    assert np.array_equal(got2["best"], orc.best)
    prob2.close()


def test_checkpoint_resume_through_noalloc(lib):
    """An anneal stopped at cycle 37 with a checkpoint and resumed, both halves through ssqa_anneal_noalloc,
    equals one uninterrupted ssqa_anneal (d = 2, so the history travels through the scratch too)."""
    import torch
    _note("case noalloc checkpoint/resume N=200 R=8 T=9 SC=80")
    h, J = random_ising(200, 8, h_max=60, j_max=7)
    rng = np.random.default_rng(8)
    q = rng.integers(-6, 7, size=80)
    i0 = rng.integers(6, 100, size=80)
    prob = lib.Problem(h, J)
    kw = dict(replicas=8, trials=9, cycles=80, jperp=q, i0=i0, alpha=2, noise_amp=9, delay=2, seed=21,
              trace=True, final_is=True)
    full = lib.ssqa_anneal(prob, **kw)
    torch.cuda.synchronize()
    first = lib.ssqa_anneal_noalloc(prob, stop_cycle=37, checkpoint=True, **kw)
    torch.cuda.synchronize()
    state = first.checkpoint
    assert state.cycle == 37
    first.checkpoint = None
    second = lib.ssqa_anneal_noalloc(prob, resume=state, out=first, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(second.best_energy.cpu().numpy(), full.best_energy.cpu().numpy())
    assert np.array_equal(second.first_hit.cpu().numpy(), full.first_hit.cpu().numpy())
    assert np.array_equal(second.final_is.cpu().numpy(), full.final_is.cpu().numpy())
    assert np.array_equal(second.energy_trace.cpu().numpy(), full.energy_trace.cpu().numpy())
    prob.close()


def test_oversize_state_is_refused(lib):
    """GI n = 50 (N = 2500), R = 64, T = 1024 needs about 190 MB of device state: refused with SSQA_ENOTSUP
    and a message naming the limit, before any device work; the same anneal with T = 8 fits and runs."""
    import torch
    _note("case noalloc oversize refused")
    h, J, e_star = gi_case(50, 2)
    q, i0, noise = paper_schedules(20, tau=5)
    prob = lib.Problem(h, J)
    kw = dict(replicas=64, cycles=20, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=0, target=e_star)
    with pytest.raises(lib.SSQAError) as err:
        lib.ssqa_anneal_noalloc(prob, trials=1024, **kw)
    assert err.value.name == "SSQA_ENOTSUP" and "fixed scratch" in str(err.value)
    got, ref = _both(lib, prob, trials=8, trace=True, **kw)
    _equal(got, ref)
    torch.cuda.synchronize()
    prob.close()
