"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C source is compiled with -fsanitize=address,undefined (every
undefined-behaviour report fatal) into a separate library, and the non-slow
pins of test_oracle_pins.py run against it in a child interpreter with the
ASan runtime loaded first.  An out-of-bounds access, use after free, signed
overflow, misaligned or null access, or shift out of range in the oracle ends
that run with a report, and this test fails.  CPU only.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's ASan runtime is not installed")
def test_oracle_pins_clean_under_asan_and_ubsan(tmp_path):
    so = oracle.compile_variant(
        oracle.source(), str(tmp_path / "liboracle_asan.so"),
        extra_flags=("-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                     "-fno-omit-frame-pointer", "-g"))
    env = dict(os.environ)
    env["RMP_ORACLE_LIB"] = so
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = _runtime("libasan.so") + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    cmd = [sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"),
           "-q", "-x", "-m", "not slow and not gpu", "-p", "no:cacheprovider"]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
