"""The oracle's pin and brute-force tests with oracle.c built under
AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal), so
that an out-of-bounds access, a use after free or an overflow in the
reference simulator fails the run instead of passing silently.  CPU only.
"""
import os
import subprocess
import sys

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pins_and_brute_force_under_sanitizers(tmp_path):
    lib = oracle.compile_oracle(os.path.join(ROOT, "oracle", "oracle.c"), str(tmp_path / "liboracle_san.so"),
                                sanitize=True)
    env = dict(os.environ, GATESIM_ORACLE_LIB=lib, LD_PRELOAD=oracle.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle_pins.py", "tests/test_oracle_brute.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
