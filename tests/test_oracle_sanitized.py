"""The oracle's CPU tests against its AddressSanitizer + UBSan build
(oracle/run_sanitized_tests.py): no out-of-bounds access, use after free or
undefined behaviour in the C oracle on any pinned case."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc with its sanitizer runtimes")
def test_oracle_under_address_and_ub_sanitizers():
    if os.environ.get("VOXLOD_ORACLE_SANITIZE") == "1":
        pytest.skip("already inside the sanitized run")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "oracle", "run_sanitized_tests.py")], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
