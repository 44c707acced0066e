"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc) runs the pins against itself: an out-of-bounds index, a use after
free, a signed overflow or a bad shift anywhere in its hand-written index
arithmetic (the CSR fills, the shed stack, the level blocks, the u128
stability sums) stops the run instead of passing silently. The pins run in a
child process with the sanitizer runtime preloaded and the instrumented build
selected through CE_ORACLE_LIB."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ce_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_causal.py", "tests/test_oracle_discrete.py",
        "tests/test_oracle_hyper.py", "tests/test_oracle_levels.py"]


@pytest.mark.slow
@pytest.mark.timeout(1500)
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-shared", "-fPIC", "-o", str(lib), SRC])
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, CE_ORACLE_LIB=str(lib), LD_PRELOAD=(asan + " " + pre).strip(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=1400)
    tail = r.stdout[-4000:] + "\n" + r.stderr[-4000:]
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
    assert " passed" in r.stdout, tail
