"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

api.cpp, host.cpp, server.cpp and tune.cpp (the C ABI's argument checks, the schedules, the graph-isomorphism
mapping, the server's submit path, the autotuner's cache reader) and work_order.hpp are compiled for the host
only with -fsanitize=address,undefined (no recovery from undefined behaviour) and linked with the kernels'
regular objects into tests/sanitize_host_check.cpp, which drives every path that runs without a device.  A sanitizer report aborts
the program, so the test passes only on a clean run that prints "ok"."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2302_12454_amd")
CSRC = os.path.join(PKG, "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_under_asan_and_ubsan(tmp_path):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    kernels = [os.path.join(PKG, "_build", f) for f in ("sweep.o", "sa.o")]
    if not all(os.path.exists(k) for k in kernels):
        from paper_2302_12454_amd import build as b
        b.build()
    objs = []
    common = ["-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SAN]
    for src in ("api.cpp", "host.cpp", "server.cpp", "tune.cpp"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([cc, *common, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-c",
                        os.path.join(CSRC, src), "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    drv = str(tmp_path / "drv.o")
    subprocess.run([cc, *common, "-c", os.path.join(ROOT, "tests", "sanitize_host_check.cpp"), "-o", drv],
                   check=True, capture_output=True)
    exe = str(tmp_path / "sanitize_host_check")
    subprocess.run([cc, *SAN, "--offload-arch=gfx950", drv, *objs, *kernels, "-o", exe], check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout[-3000:] + res.stderr[-3000:]
