"""Pins for the oracle's Philox4x32-10 and its stream layout (CPU only)."""

import json
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def _h(s):
    return int(s, 16)


def test_known_answer_vectors():
    """Published Random123 known-answer vectors (golden file cites the source)."""
    with open(GOLDEN) as f:
        kat = json.load(f)["vectors"]
    for v in kat:
        c = [_h(x) for x in v["ctr"]]
        k = [_h(x) for x in v["key"]]
        out = philox.philox4x32_10(*c, *k)
        assert [int(o) for o in out] == [_h(x) for x in v["out"]]


ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
struct P : rocrand_device::philox4x32_10_engine {
  uint4 tr(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main(int argc, char** argv) {
  P e;
  unsigned a[6];
  while (scanf("%u %u %u %u %u %u", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
    uint4 r = e.tr(uint4{a[0], a[1], a[2], a[3]}, uint2{a[4], a[5]});
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_host_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header or hipcc not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "p.hip"
    src.write_text(ROCRAND_PROG)
    exe = d / "p"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    return str(exe)


def test_against_rocrand_header(rocrand_host_philox):
    """An independent Philox4x32-10 (rocRAND's open-source header, run on the host)."""
    rng = np.random.default_rng(7)
    vals = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    vals[:5, :4] = [[0, 0, 0, 0], [1, 2, 3, 4], [7, 0, 63, 1023], [2000, 19, 25, 511], [1, 0, 0, 0]]
    inp = "\n".join(" ".join(str(int(x)) for x in row) for row in vals) + "\n"
    res = subprocess.run([rocrand_host_philox], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in line.split()] for line in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    ours = np.stack(philox.philox4x32_10(vals[:, 0], vals[:, 1], vals[:, 2], vals[:, 3],
                                         vals[:, 4], vals[:, 5]), axis=1)
    assert np.array_equal(ours, ref)


def test_stream_layout_against_single_calls():
    """Spin i of replica k, trial b, tag t takes bit (i & 31) of word (i & 127) >> 5
    of Philox(counter = (t, i >> 7, k, b), key = seed halves)."""
    seed = 0x123456789ABCDEF0
    bits = philox.stream_bits(seed, 5, 300, [0, 3], [0, 9])
    for bi, b in enumerate([0, 9]):
        for ki, k in enumerate([0, 3]):
            for i in [0, 1, 31, 32, 63, 64, 127, 128, 129, 255, 256, 299]:
                out = philox.philox4x32_10(5, i >> 7, k, b, seed & 0xFFFFFFFF, seed >> 32)
                word = int(out[(i & 127) >> 5])
                assert bits[bi, ki, i] == (word >> (i & 31)) & 1


def test_stream_subset_consistency_and_balance():
    full = philox.stream_bits(3, 17, 2500, 8, 6)
    sub = philox.stream_bits(3, 17, 2500, [2, 5], [4])
    assert np.array_equal(full[4][[2, 5]], sub[0])
    frac = full.mean()
    assert abs(frac - 0.5) < 0.01
    # different tags and seeds give different streams
    assert not np.array_equal(full, philox.stream_bits(3, 18, 2500, 8, 6))
    assert not np.array_equal(full, philox.stream_bits(4, 17, 2500, 8, 6))
