"""The FP64 reference built with the undefined-behaviour sanitizer (host
code, gcc; any report aborts) passes all of its pins: no out-of-range
shifts, signed overflow, misaligned or null accesses in the reference the
GPU path is judged against."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_grad.py", "tests/test_oracle_oit.py",
        "tests/test_oracle_sorted.py", "tests/test_oracle_earlyout.py"]


def test_reference_pins_pass_under_ubsan(tmp_path):
    lib = tmp_path / "liboracle.so"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fsanitize=undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas", "-o", str(lib),
           os.path.join(ROOT, "oracle", "wsr_oracle.c"), "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0:
        pytest.skip("gcc cannot build with -fsanitize=undefined here: " + b.stderr[-300:])
    env = dict(os.environ, WSR_ORACLE_LIB=str(lib), UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "runtime error" not in r.stderr
