"""The host code (plan, engine, C ABI) under AddressSanitizer and
UndefinedBehaviorSanitizer: the sanitizer build of the library runs the
plan-parity and ABI tests in a child process on the CPU; any report aborts
that process and fails this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_plan_and_abi_under_sanitizers():
    from paper_1510_07087_amd import build as B
    lib = B.build_sanitized()
    env = B.sanitizer_env()
    assert env["DH2_LIBRARY"] == lib
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_plan_parity.py"),
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out
