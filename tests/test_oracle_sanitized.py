"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The FP64 oracle is the checker every parity claim rests on, so its own
memory safety is tested: the same source is built with
`-fsanitize=address,undefined` and the oracle's pin tests, its adjoint
finite-difference checks, the cell-type pins and the APD90 pins run against
that build in a child interpreter with the sanitizer runtimes preloaded.  Any
out-of-bounds access, use after free or undefined arithmetic (signed
overflow, bad shifts, misaligned loads) ends the child with the sanitizer's
exit code and a report, and fails this test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_celltypes.py",
                "tests/test_oracle_apd.py", "tests/test_adjoint_cpu.py",
                "tests/test_oracle_fibrosis.py", "tests/test_oracle_time_pins.py",
                "tests/test_oracle_tp06_balance.py", "tests/test_oracle_tp06_properties.py"]


def test_oracle_tests_pass_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    ob.build(sanitize=True)
    env = ob.sanitizer_env()
    # the library's host-side model code is not part of the oracle; the
    # tests that call it load the GPU library and stay out of this run
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           "-m", "not gpu", "-k", "not library_substep_vjp and not kernel_tp06_code"] + ORACLE_TESTS
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-6000:] + "\n" + r.stderr[-6000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out
    assert r.returncode == 0, out
    assert " passed" in r.stdout, out
