"""The oracle's CPU pins, run against a build of the same oracle source with
gcc's AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's exact sums use word-indexed big-integer arithmetic (shifted limb
adds, bit-by-bit rounding); an index one word past a limb array or a shift by
the word width would not change most results but is exactly what these
sanitizers report. The pins run in a child interpreter with the sanitizer
runtimes preloaded and the instrumented library selected through
MMLTTB_ORACLE_LIB; any report fails the child (halt on the first error).
The mutant tests are left out: they compile variants of their own.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mmlttb_oracle.c")
PIN_FILES = [
    "tests/test_oracle_pins.py",
    "tests/test_oracle_downsamplers.py",
    "tests/test_oracle_typed.py",
    "tests/test_oracle_simplifiers.py",
    "tests/test_fig3_example.py",
]


def _runtime(name: str) -> str | None:
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout
    except (OSError, subprocess.CalledProcessError):
        return None
    p = p.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_pass_under_address_and_ub_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-Wall", "-Werror", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-o", lib, SRC, "-lm"])
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": f"{asan}:{ubsan}",
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
        "MMLTTB_ORACLE_LIB": lib,
    })
    res = subprocess.run([sys.executable, "-m", "pytest", *PIN_FILES, "-x", "-q", "-m", "not gpu",
                          "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, f"sanitized oracle pins failed (rc {res.returncode}):\n{tail}"
    assert "passed" in res.stdout and "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, tail
