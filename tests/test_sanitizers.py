"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The oracle (oracle/oracle.c) is built with -fsanitize=address,undefined and the whole pin
  battery runs on it in a child Python process with the sanitizer runtimes preloaded, so every
  oracle routine the pins reach (all of them, batched forms included) is checked for
  out-of-bounds accesses, use after free and undefined arithmetic.
* The library's host table builder (csrc/tables.cpp: the exact B_n recurrence in __int128, the
  swap matrices of both sides, the z coefficients, every packed and fragment layout built at
  context creation) is built the same way with a driver (tests/sanitize/tables_check.cpp)
  that checks the swap identities.
* A planted one-element overflow in a copy of the oracle must abort the pin run, which shows
  that the sanitizer is active in these builds.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_SRC = os.path.join(ROOT, "oracle", "oracle.c")
CSRC = os.path.join(ROOT, "paper_2202_02847_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc/g++ with the sanitizer runtimes")


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not installed")
    return path


def _build_oracle(src, out):
    subprocess.run(["gcc", *SAN, "-fopenmp", "-fPIC", "-shared", "-std=c99", src, "-o", out, "-lm"], check=True)


PIN_RUNNER = """
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle
from oracle_pins import PINS
o = oracle.Oracle("double", path={lib!r})
bad = [p.__name__ for p in PINS if not (lambda eb: eb[0] <= eb[1])(p(o))]
print("pins failed:", bad)
sys.exit(1 if bad else 0)
"""


def _run_pins(lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = " ".join([_runtime("libasan.so"), _runtime("libubsan.so")])
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    code = PIN_RUNNER.format(root=ROOT, tests=HERE, lib=lib)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)


def test_oracle_pins_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        _build_oracle(ORACLE_SRC, lib)
        res = _run_pins(lib)
        assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
        assert "pins failed: []" in res.stdout
        assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]


def test_planted_overflow_is_reported():
    """One element written past the regular harmonics' array: the sanitized pin run must fail."""
    text = open(ORACLE_SRC).read()
    old = "memset(R, 0, sizeof(real) * (size_t)P * (P + 1));"
    assert old in text
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "oracle_overflow.c")
        open(src, "w").write(text.replace(old, "memset(R, 0, sizeof(real) * ((size_t)P * (P + 1) + 1));", 1))
        lib = os.path.join(d, "liboracle_overflow.so")
        _build_oracle(src, lib)
        res = _run_pins(lib)
        assert res.returncode != 0 and "AddressSanitizer" in res.stderr, res.stderr[-2000:]


def test_table_builder_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tables_check")
        subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
                        os.path.join(CSRC, "tables.cpp"), os.path.join(HERE, "sanitize", "tables_check.cpp"),
                        "-o", exe], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr[-4000:]
        assert "tables_check: 0 failures" in res.stdout
