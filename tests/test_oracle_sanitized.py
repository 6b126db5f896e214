"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A copy of the oracle's C sources is built with gcc -fsanitize=address,
undefined (host code only, no GPU code involved) and the pins of the single-
phase and multiphase oracles run against it in a child process
(``STEV_ORACLE_LIB``), with the ASan runtime preloaded into the Python
interpreter.  Any out-of-bounds access, use after free or undefined
operation aborts the child and fails the test."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no ASan runtime for gcc here")
    for f in ("stev_oracle.c", "c3m_oracle.c", "stev_oracle.h"):
        shutil.copy(os.path.join(ROOT, "oracle", f), tmp_path)
    lib = os.path.join(tmp_path, "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", lib, os.path.join(tmp_path, "stev_oracle.c"),
                           os.path.join(tmp_path, "c3m_oracle.c"), "-lm"])
    env = dict(os.environ, STEV_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_c3m.py"),
                        "-k", "not convergence_to_radau and not t11"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    print(r.stdout.strip().splitlines()[-1] if r.stdout.strip() else "(no output)")
    assert r.returncode == 0, tail
    assert " passed" in r.stdout, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
