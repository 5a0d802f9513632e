"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C++) built with -fsanitize=address,undefined runs the
  oracle's own test files in a child process with gcc's sanitizer runtimes
  preloaded: every pin and property test, no report allowed (UBSan aborts on
  its first finding).
* The HIP library built with the sanitizers on its host code only (argument
  validation, model tables, launch planning, the server's bookkeeping) runs the
  ABI tests the same way with clang's ASan runtime.

Each child first checks that the sanitized build is the library it loaded."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_TESTS = ["test_oracle_costs.py", "test_oracle_dynamics.py", "test_oracle_forced.py", "test_oracle_mppi.py",
                "test_oracle_noise.py", "test_oracle_spline.py", "test_oracle_spline_variants.py",
                "test_oracle_tasks.py", "test_oracle_warmstart.py"]

CHECK_ORACLE = """
import oracle as O
O.lib()
maps = open('/proc/self/maps').read()
assert 'liboracle_san.so' in maps and 'libasan' in maps, 'sanitized oracle not loaded'
"""

CHECK_MPPI = """
from paper_2511_19204_amd import mppi
mppi.lib()
maps = open('/proc/self/maps').read()
assert 'libmppi_san.so' in maps and 'libclang_rt.asan' in maps, 'sanitized library not loaded'
"""


def _run(env, args, timeout):
    res = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return res.returncode, res.stdout[-3000:] + res.stderr[-3000:]


def test_oracle_under_asan_and_ubsan():
    from oracle import build
    lib = build.build(force=False, sanitize=True)
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=":".join(build.sanitizer_runtimes()),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out = _run(env, ["-c", CHECK_ORACLE], 120)
    assert rc == 0, out
    rc, out = _run(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                         *[os.path.join("tests", t) for t in ORACLE_TESTS]], 600)
    assert rc == 0, out
    assert "passed" in out and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out


def test_host_runtime_under_asan_and_ubsan():
    from paper_2511_19204_amd import build
    try:
        lib = build.build(force=False, sanitize=True)
    except RuntimeError as e:  # pragma: no cover - reported, not hidden
        pytest.fail(f"host-sanitizer build failed: {e}")
    rt = build.sanitizer_runtime()
    env = dict(os.environ, MPPI_LIB=lib, LD_PRELOAD=rt, LD_LIBRARY_PATH=os.path.dirname(rt),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out = _run(env, ["-c", CHECK_MPPI], 120)
    assert rc == 0, out
    rc, out = _run(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                         os.path.join("tests", "test_abi.py")], 600)
    assert rc == 0, out
    assert "passed" in out and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
