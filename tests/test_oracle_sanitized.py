"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only), running its own pins: an out-of-bounds access, a use after
free, a signed overflow or a bad shift anywhere in the oracle's code paths that
the pins reach stops the child run.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pcpic_oracle.c")

pytestmark = pytest.mark.slow


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "oracle"), "-o", lib, SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    pre = " ".join(p for p in (asan, ubsan, os.environ.get("LD_PRELOAD", "")) if p)
    log = str(tmp_path / "san")
    env = dict(os.environ, PCPIC_ORACLE_LIB=lib, LD_PRELOAD=pre,
               ASAN_OPTIONS=f"detect_leaks=0:abort_on_error=1:log_path={log}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={log}")
    tests = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_pins.py", "test_oracle_adjoint.py",
                                                     "test_oracle_parallel.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = "".join(open(os.path.join(tmp_path, f)).read() for f in sorted(os.listdir(tmp_path))
                      if f.startswith("san"))
    tail = (r.stdout + r.stderr)[-2000:] + reports[:3000]
    assert r.returncode == 0 and not reports, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
