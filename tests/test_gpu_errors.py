"""GPU tests of ssqa_anneal's argument checks through the C ABI: every rejected argument gives its status
and a message naming the argument, launches nothing, and leaves the library able to run a valid anneal
that still equals the oracle bit for bit."""

import sys

import numpy as np
import pytest

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


SC = 10


def _base():
    q, i0, noise = paper_schedules(SC, tau=4)
    return dict(replicas=8, trials=4, cycles=SC, jperp=np.array(q), i0=np.array(i0), alpha=1, noise_amp=noise,
                delay=1, seed=0)


def _bad_i0(value, at):
    i0 = _base()["i0"].copy()
    i0[at] = value
    return i0


def _bad_jperp(value, at):
    q = _base()["jperp"].copy()
    q[at] = value
    return q


# (name, changes to the valid arguments, expected status, text the message must contain)
CASES = [
    ("replicas 0", dict(replicas=0), "SSQA_EINVAL", "replicas"),
    ("trials 0", dict(trials=0), "SSQA_EINVAL", "trials"),
    ("cycles -1", dict(cycles=-1), "SSQA_EINVAL", "cycles"),
    ("block_columns 96", dict(block_columns=96), "SSQA_EINVAL", "block_columns"),
    ("replicas beyond the block", dict(replicas=65, block_columns=64), "SSQA_ENOTSUP", "exceeds"),
    ("delay 7", dict(delay=7), "SSQA_EINVAL", "delay"),
    ("delay -1", dict(delay=-1), "SSQA_EINVAL", "delay"),
    ("alpha 0", dict(alpha=0), "SSQA_EINVAL", "alpha"),
    ("noise_amp -1", dict(noise_amp=-1), "SSQA_EINVAL", "noise_amp"),
    ("noise_amp 2^20 + 1", dict(noise_amp=(1 << 20) + 1), "SSQA_EINVAL", "noise_amp"),
    ("coupling_mode 2", dict(coupling_mode=2), "SSQA_EINVAL", "coupling_mode"),
    ("cycles_per_launch -1", dict(cycles_per_launch=-1), "SSQA_EINVAL", "cycles_per_launch"),
    ("i0 below alpha", dict(i0=_bad_i0(0, 3)), "SSQA_EINVAL", "i0[3]"),
    ("i0 above 127", dict(i0=_bad_i0(128, 9)), "SSQA_EINVAL", "i0[9]"),
    ("i0 below alpha = 3", dict(alpha=3, i0=_bad_i0(2, 0)), "SSQA_EINVAL", "i0[0]"),
    ("jperp beyond 2^20", dict(jperp=_bad_jperp((1 << 20) + 1, 5)), "SSQA_EINVAL", "jperp[5]"),
    ("jperp below -2^20", dict(jperp=_bad_jperp(-(1 << 20) - 1, 0)), "SSQA_EINVAL", "jperp[0]"),
    ("operand_format 3", dict(operand_format=3), "SSQA_EINVAL", "operand_format"),
    ("operand_format -1", dict(operand_format=-1), "SSQA_EINVAL", "operand_format"),
]


@pytest.fixture(scope="module")
def problems(lib):
    h, J, e_star = gi_case(5, 0)                      # N = 25, every J entry exact in fp4
    hi, Ji = random_ising(40, 2, h_max=30, j_max=11)  # entries such as 5 and 7: int8 operands only
    hp, Jp = random_ising(40, 3, h_max=30, j_max=500)  # |J| beyond 127: two int8 planes
    return (lib.Problem(h, J), h, J, e_star), lib.Problem(hi, Ji), lib.Problem(hp, Jp)


@pytest.mark.parametrize("name,change,status,text", CASES, ids=[c[0] for c in CASES])
def test_anneal_rejects(lib, problems, name, change, status, text):
    _note(f"case rejected argument: {name}")
    prob = problems[0][0]
    kw = dict(_base(), **change)
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_anneal(prob, **kw)
    assert ei.value.name == status
    assert text in str(ei.value), str(ei.value)


def test_fp4_only_requests_on_int8_problem(lib, problems):
    """fp4 operands on a J without fp4 codes are refused; 128 columns with int8 operands are refused only
    when J needs more than one int8 plane."""
    _note("case fp4-only requests on an int8 problem")
    prob = problems[1]
    assert not prob.fp4_exact and prob.planes == 1
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_anneal(prob, **dict(_base(), operand_format=2))
    assert ei.value.name == "SSQA_ENOTSUP" and "fp4" in str(ei.value), str(ei.value)
    two = problems[2]
    assert two.planes == 2
    with pytest.raises(lib.SSQAError) as ei:
        lib.ssqa_anneal(two, **dict(_base(), block_columns=128))
    assert ei.value.name == "SSQA_ENOTSUP" and "one int8 plane" in str(ei.value), str(ei.value)


def test_batch_rejects_a_bad_job(lib, problems):
    _note("case batch with one rejected job")
    prob = problems[0][0]
    good = _base()
    bad = dict(_base(), alpha=0)
    with pytest.raises(lib.SSQAError) as ei:
        lib.Batch([(prob, good), (prob, bad)])
    assert ei.value.name == "SSQA_EINVAL" and "alpha" in str(ei.value)


def test_valid_anneal_after_rejections(lib, problems):
    """After every rejection above, a valid anneal on the same problem still equals the oracle."""
    _note("case valid anneal after rejections")
    prob, h, J, e_star = problems[0]
    q, i0, noise = paper_schedules(SC, tau=4)
    kw = dict(replicas=8, trials=4, cycles=SC, q=q, i0=i0, alpha=1, noise=noise, delay=1, seed=0, target=e_star)
    assert_same(run_gpu(prob, **kw), run_oracle(h, J, **kw))
