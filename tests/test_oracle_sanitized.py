"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs every pin in a child process: no memory error, no
undefined behaviour, and every pin still holds."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gcp_oracle.c")

DRIVER = r"""
import sys
import oracle
import pins
print("oracle library:", oracle.lib()._name, flush=True)
failed = [n for n in sorted(pins.ALL_PINS) if not pins.ALL_PINS[n]()[0]]
print("pins run:", len(pins.ALL_PINS), "failed:", failed, flush=True)
sys.exit(1 if failed else 0)
"""


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_pins_under_address_and_undefined_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", lib, SRC, "-lm"])
    env = dict(os.environ)
    # the sanitizer runtime must come first among the loaded libraries;
    # anything already preloaded stays after it
    env["LD_PRELOAD"] = asan + ((":" + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["GCP_ORACLE_LIB"] = lib
    env["PYTHONPATH"] = os.pathsep.join([ROOT, os.path.join(ROOT, "tests")])
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True, timeout=900)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert f"oracle library: {lib}" in r.stdout
    assert "failed: []" in r.stdout
