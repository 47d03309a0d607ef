"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the C
source is rebuilt with both (every report fatal) and the oracle's pins run
against that build in a child process with libasan preloaded.  Any
out-of-bounds access, use after free or undefined behaviour in the oracle
fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env.update({"ORACLE_LIB": lib, "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    pins = ["tests/test_oracle_pins.py", "tests/test_oracle_flag_pins.py", "tests/test_oracle_aa_pins.py",
            "tests/test_oracle_lens_pins.py", "tests/test_oracle_prim_pins.py"]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]
                         + pins, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "passed" in res.stdout and "AddressSanitizer" not in tail and "runtime error" not in tail, tail
