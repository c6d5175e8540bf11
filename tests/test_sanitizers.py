"""The host-side native code under the address and undefined-behaviour
sanitizers: the CPU oracle (oracle.c), the multi-threaded CPU baseline
(scantrans.c) and the input generator (gen.cpp) are built instrumented
(MGT_HOST_SANITIZE=1) and the CPU test suites that drive them run against
those builds in a child process that preloads the sanitizer runtime. Any
report (an out-of-bounds access, a use after free, undefined behaviour) fails
the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUITES = ["tests/test_oracle.py", "tests/test_values_oracle.py", "tests/test_views_oracle.py",
          "tests/test_symmetric_oracle.py", "tests/test_scantrans_baseline.py"]


def _runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_host_code_under_sanitizers():
    asan = _runtime()
    if asan is None:
        pytest.skip("no address-sanitizer runtime for gcc on this host")
    env = dict(os.environ, MGT_HOST_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HYPOTHESIS_PROFILE=os.environ.get("HYPOTHESIS_PROFILE", ""))
    code = ("import sys; sys.path.insert(0, '.'); "
            "from workloads import gen; import oracle; gen.build(force=True); "
            "oracle.build(force=True)")
    b = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *SUITES], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
