"""GPU tests of checkpoint / resume: an anneal stopped at cycle t1 and resumed from its checkpoint (even
under another tiling) equals the uninterrupted anneal bit for bit, and the checkpoint equals the oracle's
state at t1 (counters and delayed spins)."""

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


def _unpack(history, n):
    """int32 [T, R, d, W] bit-packed spins -> int8 [T, R, d, N] of +-1."""
    h = history.cpu().numpy().view(np.uint32)
    bits = (h[..., None] >> np.arange(32, dtype=np.uint32)) & 1
    bits = bits.reshape(*h.shape[:-1], h.shape[-1] * 32)[..., :n]
    return np.where(bits == 1, 1, -1).astype(np.int8)


def _case(name):
    if name == "gi6_fp4":
        h, J, e_star = gi_case(6, 3)
        q, i0, noise = paper_schedules(300, tau=25)
        kw = dict(replicas=8, trials=20, cycles=300, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=1, seed=4,
                  target=e_star)
        return h, J, kw, 150, (0, 0)
    if name == "gi6_wide_to_narrow":
        h, J, e_star = gi_case(6, 5)
        q, i0, noise = paper_schedules(120, tau=20)
        kw = dict(replicas=16, trials=24, cycles=120, jperp=q, i0=i0, alpha=1, noise_amp=noise, delay=2, seed=6,
                  target=e_star)
        return h, J, kw, 70, (128, 64)
    if name == "ising300_d2_mode1":
        h, J = random_ising(300, 21, h_max=70, j_max=9)
        rng = np.random.default_rng(21)
        q = rng.integers(-6, 7, size=60)
        i0 = rng.integers(4, 90, size=60)
        kw = dict(replicas=5, trials=13, cycles=60, jperp=q, i0=i0, alpha=3, noise_amp=11, delay=2, seed=21,
                  coupling_mode=1)
        return h, J, kw, 25, (64, 32)
    h, J = random_ising(129, 22, h_max=50, j_max=6)
    rng = np.random.default_rng(22)
    q = rng.integers(0, 8, size=40)
    i0 = rng.integers(3, 60, size=40)
    kw = dict(replicas=7, trials=9, cycles=40, jperp=q, i0=i0, alpha=1, noise_amp=7, delay=0, seed=22)
    return h, J, kw, 17, (0, 0)


@pytest.mark.parametrize("name", ["gi6_fp4", "gi6_wide_to_narrow", "ising300_d2_mode1", "ising129_d0"])
def test_checkpoint_resume_equals_uninterrupted(lib, name):
    import torch
    _note(f"case checkpoint/resume {name}")
    h, J, kw, t1, (bc1, bc2) = _case(name)
    prob = lib.Problem(h, J)
    full = lib.ssqa_anneal(prob, trace=True, final_is=True, **kw)
    first = lib.ssqa_anneal(prob, trace=True, final_is=True, stop_cycle=t1, checkpoint=True, block_columns=bc1,
                            **kw)
    torch.cuda.synchronize()
    state = first.checkpoint
    assert state.cycle == t1
    # the checkpoint is the oracle's state after t1 cycles
    ref = run_oracle(h, J, replicas=kw["replicas"], trials=kw["trials"], cycles=t1, q=kw["jperp"], i0=kw["i0"],
                     alpha=kw["alpha"], noise=kw["noise_amp"], delay=kw["delay"], seed=kw["seed"],
                     mode=kw.get("coupling_mode", 0), target=kw.get("target"))
    assert np.array_equal(state.counters.cpu().numpy(), ref.Is)
    d = kw["delay"]
    if d > 0:
        spins = _unpack(state.history, len(h))
        for s in range(1, d + 1):
            assert np.array_equal(spins[:, :, s - 1, :], ref.state.history[s]), s
    else:
        assert state.history is None
    # resume into the same outputs (best energies and first hits carry over), under another tiling
    first.checkpoint = None
    second = lib.ssqa_anneal(prob, resume=state, out=first, block_columns=bc2, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(second.energy_trace.cpu().numpy(), full.energy_trace.cpu().numpy())
    assert np.array_equal(second.best_energy.cpu().numpy(), full.best_energy.cpu().numpy())
    assert np.array_equal(second.first_hit.cpu().numpy(), full.first_hit.cpu().numpy())
    assert np.array_equal(second.final_is.cpu().numpy(), full.final_is.cpu().numpy())


def test_resume_argument_errors(lib):
    h, J, kw, t1, _ = _case("ising129_d0")
    prob = lib.Problem(h, J)
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_anneal(prob, stop_cycle=kw["cycles"] + 1, **kw)
    assert ei.value.name == "SSQA_EINVAL"
    first = lib.ssqa_anneal(prob, stop_cycle=t1, checkpoint=True, **kw)
    st = first.checkpoint
    with pytest.raises(lib.SSQAError):
        bad = lib.AnnealState(counters=st.counters, history=None, cycle=kw["cycles"] + 5)
        lib.ssqa_anneal(prob, resume=bad, **kw)
