"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle's pin tests run in a child process against a sanitized build of
hm_oracle.c (HM_ORACLE_SANITIZE=1), with the sanitizer runtime preloaded into
the interpreter; any report (out-of-bounds access, use after free, signed
overflow, misaligned load, ...) stops the child with a failure."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not available")
    env = dict(os.environ)
    env.update({
        "HM_ORACLE_SANITIZE": "1",
        "LD_PRELOAD": f"{asan}:{ubsan}",
        # the interpreter itself is not instrumented: no leak report at exit
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    tests = ["tests/test_oracle_raster.py", "tests/test_oracle_lod_gen.py",
             "tests/test_oracle_resolve.py", "tests/test_oracle_readings.py",
             "tests/test_oracle_gbuf.py", "tests/test_oracle_dom.py",
             "tests/test_oracle_threads.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    log = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in log, log[-4000:]
    assert "runtime error:" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
