"""Runs the oracle's CPU tests against a build of oracle.c with
AddressSanitizer and UndefinedBehaviorSanitizer.

    python oracle/run_sanitized_tests.py [extra pytest arguments]

The sanitized library (oracle/liboracle_san.so, gcc, host code only) is built
first; the tests then run in a child process with VOXLOD_ORACLE_SANITIZE=1 and
libasan preloaded into the Python interpreter (which is not itself built with
the sanitizer, so leak checking is off).  Any out-of-bounds access, use after
free or undefined behaviour in the oracle aborts the run with a report.
Exits with the tests' status.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TESTS = ["tests/test_oracle_pins.py", "tests/test_golden_and_inputs.py"]


def main() -> int:
    env = dict(os.environ)
    env["VOXLOD_ORACLE_SANITIZE"] = "1"
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT, env=env, check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    env["LD_PRELOAD"] = " ".join([asan, ubsan] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else []))
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *TESTS,
           *sys.argv[1:]]
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main())
