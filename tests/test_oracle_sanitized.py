"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

The C oracle is built a second time with -fsanitize=address,undefined (every
report fatal) and the pin suites of the C oracle run against that build in a
child process with the ASan runtime preloaded.  An out-of-bounds access, a
use of freed memory, a signed overflow or a misaligned load anywhere on the
paths the pins exercise ends the child with a report and fails this test.
CPU only.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as oracle_build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PIN_SUITES = ["test_oracle_models.py", "test_oracle_tableau.py", "test_oracle_variants.py",
              "test_oracle_lyapunov.py", "test_oracle_controller.py"]


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                           text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_pass_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle_build.build(sanitize=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ORACLE_LIB=lib,
               OMP_NUM_THREADS="4")
    # the child really maps the sanitized build
    probe = subprocess.run(
        [sys.executable, "-c",
         "import oracle; oracle.lib(); import sys; "
         "sys.exit(0 if 'liboracle_san.so' in open('/proc/self/maps').read() else 3)"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
         *[os.path.join(HERE, s) for s in PIN_SUITES]],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
