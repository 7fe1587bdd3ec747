"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) passes its pins: every out-of-bounds access, use
after free, signed overflow, misaligned or null access and shift out of
range in the C code aborts the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lcd_oracle.c")

# pins that drive every entry point of the oracle library: growth and sweep,
# merge phase, seed selection, NMI, the specified log
PINS = ["tests/test_oracle_log.py", "tests/test_oracle_bruteforce.py", "tests/test_oracle_replay.py",
        "tests/test_oracle_limits.py", "tests/test_oracle_merge.py", "tests/test_oracle_seeds.py",
        "tests/test_oracle_nmi.py"]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=%s" % name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    so = tmp_path / "liblcd_oracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    SRC, "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, LCDO_LIB=str(so), LD_PRELOAD="%s:%s" % (asan, ubsan),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not slow",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, "sanitized oracle failed:\n%s\n%s" % (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
