"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
its pins without a report: out-of-bounds accesses, use after free, signed
overflow, misaligned or null accesses in fwi_oracle.c abort the child process
and fail this test.  The pins run in a child process that preloads the ASan
runtime (the interpreter itself is not instrumented; leak checking is off
because the interpreter keeps its allocations until exit)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_stencil.py", "tests/test_oracle_w2.py", "tests/test_oracle_guidance.py",
        "tests/test_oracle_baselines.py", "tests/test_oracle_pml.py::test_pml_gradient_matches_finite_differences",
        "tests/test_oracle_pml.py::test_pml_without_layer_is_the_leapfrog"]


def test_oracle_pins_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    import oracle

    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=lib, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
