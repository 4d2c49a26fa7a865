"""GPU parity at the edges of the accepted ranges: the fp4 accumulator bound (Eq. 6a-b need the field
exactly), very large noise and coupling amplitudes, and J split into three int8 planes.  Every case is
compared bit for bit with the oracle; a request the library cannot run exactly is refused."""

import sys

import numpy as np
import pytest

from synth import random_ising
from tests.parity_util import assert_same, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

FP4_LIMIT = 1 << 22          # every partial sum of the fp32 accumulation must stay below 2^22 in magnitude


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


def _fp4_model(n, seed, k=4):
    """A symmetric J with entries in {0, +-1, +-2, +-3, +-4, +-6} (exact in e2m1), small h, and row 0
    coupled by +6 to spins 1..k, so that row 0 carries the largest bound once h_0 is made large."""
    rng = np.random.default_rng(seed)
    vals = np.array([0, 0, 0, 1, -1, 2, -2, 3, -3, 4, -4, 6, -6])
    J = np.triu(rng.choice(vals, size=(n, n)), 1)
    J[0, :] = 0
    J[0, 1:k + 1] = 6
    J = J + J.T
    h = rng.integers(-50, 51, size=n)
    return h.astype(np.int64), J.astype(np.int64)


def _bound_rows(h, J):
    """max_i (|h_i| + 2 sum_j |J_ij|), the problem's part of the fp4 bound stated in ssqa.h."""
    return int((np.abs(h) + 2 * np.abs(J).sum(axis=1)).max())


@pytest.mark.parametrize("alpha,mode", [(1, 1), (3, 0)])
def test_fp4_exact_at_the_accumulator_bound(lib, alpha, mode):
    """h_0 = -H with H chosen so that B + n_rnd + (1 + mode) max|J_perp| + 128 = 2^22 - 1: fp4 is still
    taken, and every accumulator of row 0 starts about 2^22 below 1.5 * 2^23.  Trace, best, first hit and
    final counters equal the oracle.  One more unit of noise crosses the bound: the explicit fp4 request is
    refused (SSQA_ENOTSUP) and the automatic choice (int8) still equals the oracle."""
    _note(f"case fp4 bound alpha={alpha} mode={mode}")
    n, SC, R, T = 48, 40, 8, 6
    h, J = _fp4_model(n, 17 + alpha)
    rng = np.random.default_rng(5)
    q = rng.integers(-6, 7, size=SC)
    i0 = np.full(SC, 24)
    noise = 12
    slack = noise + (1 + mode) * int(np.abs(q).max()) + 128
    rest = 2 * int(np.abs(J[0]).sum())
    h[0] = -(FP4_LIMIT - 1 - slack - rest)
    assert _bound_rows(h, J) + slack == FP4_LIMIT - 1
    prob = lib.Problem(h, J)
    assert prob.fp4_exact
    kw = dict(replicas=R, trials=T, cycles=SC, q=q, i0=i0, alpha=alpha, noise=noise, delay=1, seed=9, mode=mode)
    ref = run_oracle(h, J, **kw)
    assert_same(run_gpu(prob, operand_format=2, **kw), ref)
    assert_same(run_gpu(prob, **kw), ref)
    kw1 = dict(kw, noise=noise + 1)
    with pytest.raises(lib.SSQAError) as err:
        run_gpu(prob, operand_format=2, **kw1)
    assert err.value.name == "SSQA_ENOTSUP" and "2^22" in str(err.value)
    assert_same(run_gpu(prob, **kw1), run_oracle(h, J, **kw1))


def test_fp4_refused_for_large_h(lib):
    """|h_0| = 5 * 10^6 with fp4-representable J: no fp4 copy is built (B >= 2^22), an explicit fp4
    request is refused, and the automatic path (int8 planes) equals the oracle."""
    _note("case fp4 large h")
    h, J = _fp4_model(40, 23)
    h[0] = 5_000_000
    h[7] = -4_999_999
    prob = lib.Problem(h, J)
    assert not prob.fp4_exact
    SC = 30
    q = np.resize([0, 2, 4, 6], SC)
    kw = dict(replicas=4, trials=5, cycles=SC, q=q, i0=np.full(SC, 24), alpha=1, noise=12, delay=1, seed=4)
    with pytest.raises(lib.SSQAError) as err:
        run_gpu(prob, operand_format=2, **kw)
    assert err.value.name == "SSQA_ENOTSUP"
    assert_same(run_gpu(prob, **kw), run_oracle(h, J, **kw))


@pytest.mark.parametrize("h_big,fp4_ok", [(0, True), (1_500_000, False)])
def test_largest_noise_and_coupling(lib, h_big, fp4_ok):
    """n_rnd = 2^20 and |J_perp| = 2^20 (the largest accepted) in coupling mode 1.  With small h the fp4 bound
    holds (3 * 2^20 + B + 128 < 2^22) and fp4 is exact; with |h_0| = 1.5 * 10^6 it does not, an explicit fp4
    request is refused and the automatic choice falls back to int8.  Both equal the oracle bit for bit."""
    _note(f"case n_rnd = J_perp = 2^20, h_big={h_big}")
    h, J = _fp4_model(40, 29)
    h[0] = h_big
    prob = lib.Problem(h, J)
    assert prob.fp4_exact
    SC = 30
    big = 1 << 20
    q = np.resize([big, -big, 0, big // 2], SC)
    i0 = np.resize([127, 24, 60], SC)
    kw = dict(replicas=6, trials=4, cycles=SC, q=q, i0=i0, alpha=2, noise=big, delay=2, seed=12, mode=1)
    ref = run_oracle(h, J, **kw)
    if fp4_ok:
        assert_same(run_gpu(prob, operand_format=2, **kw), ref)
    else:
        with pytest.raises(lib.SSQAError) as err:
            run_gpu(prob, operand_format=2, **kw)
        assert err.value.name == "SSQA_ENOTSUP"
    assert_same(run_gpu(prob, **kw), ref)
    assert_same(run_gpu(prob, operand_format=1, **kw), ref)


def test_three_int8_planes(lib):
    """|J| up to 10^5 (beyond int16): J is split into three balanced int8 planes, evaluated by Horner's
    rule in the K loop; every energy, best, first hit and final counter equals the oracle."""
    _note("case planes n=200 P=3")
    h, J = random_ising(200, 41, h_max=50_000, j_max=100_000, density=0.05)
    prob = lib.Problem(h, J)
    assert prob.planes == 3 and not prob.fp4_exact
    SC = 25
    rng = np.random.default_rng(8)
    q = rng.integers(-3000, 3000, size=SC)
    i0 = rng.integers(50, 128, size=SC)
    kw = dict(replicas=5, trials=9, cycles=SC, q=q, i0=i0, alpha=4, noise=20_000, delay=1, seed=21, mode=1)
    assert_same(run_gpu(prob, **kw), run_oracle(h, J, **kw))
