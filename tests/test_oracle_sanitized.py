"""The oracle's own pins run against an AddressSanitizer + UndefinedBehavior-
Sanitizer build of orc.c (CPU only, host code): an out-of-bounds access, a
use after free or undefined arithmetic in the oracle ends the run."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle.orc as orc

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        lib = orc.build(sanitize=True, path=os.path.join(tmp, "liborc_asan.so"))
        mods = ["test_oracle_bruteforce.py", "test_oracle_invariants.py", "test_oracle_tables.py",
                "test_oracle_switches.py", "test_oracle_q19.py", "test_oracle_front.py", "test_oracle_stability.py",
                "test_window_oracle.py", "test_mu_bound.py"]
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"]
                           + [os.path.join(TESTS, m) for m in mods],
                           cwd=ROOT, env=orc.sanitizer_env(lib), capture_output=True, text=True, timeout=1200)
        tail = (r.stdout + r.stderr)[-3000:]
        assert r.returncode == 0, tail
        assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
