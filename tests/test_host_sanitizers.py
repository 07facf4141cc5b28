"""The CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle and the host code of the HIP library are rebuilt with clang's
sanitizers (any report aborts the process), the ASan runtime is preloaded,
and every other `-m "not gpu"` test runs against those builds in a child
process.  A planted out-of-bounds read in an oracle call shows that the
sanitized build reports it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_RT = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"

pytestmark = pytest.mark.skipif(
    os.environ.get("VV10_SANITIZER_CHILD") == "1" or not os.path.exists(ASAN_RT),
    reason="inside the sanitizer run itself, or no clang ASan runtime")


def _env():
    import oracle
    from paper_2208_14639_amd import build
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": ":".join(x for x in (ASAN_RT, env.get("LD_PRELOAD", "")) if x),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1",
        "LD_LIBRARY_PATH": ":".join(x for x in ("/opt/rocm/llvm/lib", env.get("LD_LIBRARY_PATH", "")) if x),
        "VV10_LIBRARY": build.SAN_LIB,
        "VV10_ORACLE_LIBRARY": oracle.SAN_LIB,
        "VV10_SANITIZER_CHILD": "1",
    })
    return env


@pytest.fixture(scope="module")
def sanitized_builds():
    import oracle
    from paper_2208_14639_amd import build
    build.build(sanitize=True)
    oracle.build_sanitized()
    return _env()


def test_cpu_suite_under_asan_ubsan(sanitized_builds):
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-m", "not gpu", "-q", "-x",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=sanitized_builds,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr, tail


def test_sanitizer_reports_a_planted_overflow(sanitized_builds):
    """An oracle call whose coordinate array is one point short reads past
    its end; the sanitized oracle aborts with a heap-buffer-overflow."""
    code = ("import numpy as np, oracle\n"
            "n = 40\n"
            "rng = np.random.default_rng(0)\n"
            "c = rng.standard_normal((n - 1, 3))\n"
            "w = np.full(n, 0.1); r = np.full(n, 0.2); g = np.full(n, 0.01)\n"
            "oracle.pair_integrals(c, w, r, g, 6.0, 0.01)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=sanitized_builds,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
