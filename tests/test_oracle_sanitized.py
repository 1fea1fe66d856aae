"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
every pin without a report: no out-of-bounds access or use of freed memory, no
signed overflow, invalid shift or misaligned access on the inputs the pins use.

The sanitized library runs in a child process with the AddressSanitizer
runtime loaded first (a Python interpreter is not built with it); leak
detection is off, since the interpreter itself keeps memory until exit.
"""
import os
import subprocess
import sys

import pytest

import oracle

CHILD = r"""
import sys
sys.path[:0] = [sys.argv[1], sys.argv[2]]
import oracle, oracle_pins
lib = oracle.load(path=sys.argv[3])
for pin in oracle_pins.ALL_PINS:
    pin(lib)
print("ALL PINS PASSED")
"""


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_pins_under_address_and_undefined_sanitizers(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    so = str(tmp_path / "liboracle_sanitized.so")
    oracle.build(out=so, extra_flags=("-fsanitize=address,undefined",
                                      "-fno-sanitize-recover=undefined",
                                      "-fno-omit-frame-pointer", "-g"))
    env = dict(os.environ)
    # the runtime goes first; whatever the environment preloads already stays
    env["LD_PRELOAD"] = (asan + " " + env.get("LD_PRELOAD", "")).strip()
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    tests = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, "-c", CHILD, os.path.dirname(tests), tests, so],
                       capture_output=True, text=True, timeout=1200, env=env)
    report = r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr, report
    assert "runtime error:" not in r.stderr, report
    assert r.returncode == 0 and "ALL PINS PASSED" in r.stdout, (r.returncode, report)
