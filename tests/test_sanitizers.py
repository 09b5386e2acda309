"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code:
the oracle (oracle/gp_oracle.c, run under its own pin tests) and the
library's host C ABI (paper_2110_11226_amd/csrc/gp_host.cpp: generators,
validation, pre-draw, genetic operations, checked bit for bit against the
oracle by tests/_sanitize_host.py).  Both are built with gcc/g++ for the
CPU only; the sanitizer runtimes are preloaded into a child Python, and any
report aborts it (-fno-sanitize-recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-shared", "-fPIC"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    d = tmp_path_factory.mktemp("san")
    orc = str(d / "liboracle_san.so")
    host = str(d / "libgp_host_san.so")
    subprocess.run(["gcc", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", *SAN, "-o", orc,
                    os.path.join(ROOT, "oracle", "gp_oracle.c"), "-lm"], check=True)
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-o", host,
                    os.path.join(ROOT, "paper_2110_11226_amd", "csrc", "gp_host.cpp")], check=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan} {ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", GP_ORACLE_LIB=orc, OMP_NUM_THREADS="4",
               PYTHONPATH=ROOT)
    return env, host


def test_oracle_pins_under_sanitizers(sanitized):
    env, _ = sanitized
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_eval.py", "test_oracle_metrics.py", "test_oracle_grad.py", "test_oracle_generators.py",
              "test_oracle_mutation.py", "test_oracle_tournament.py", "test_oracle_philox.py",
              "test_oracle_condition.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *tests], env=env,
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])


def test_host_library_under_sanitizers(sanitized):
    env, host = sanitized
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "_sanitize_host.py"), host], env=env,
                       capture_output=True, text=True, cwd=os.path.join(ROOT, "tests"))
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "bit-exactly" in r.stdout
