"""The bounds-checked debug build (libpmlpic_check.so, -DPMLPIC_CHECK) runs the parity cases of
tests/checked_runs.py against the oracle with no failed check.  It runs in a process of its
own because a process loads one build of the library."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_2201_09084_amd", "libpmlpic_check.so")


def test_checked_build_runs_the_parity_cases():
    assert os.path.exists(LIB), "build the checked library with __graft_entry__.build()"
    env = dict(os.environ, PMLPIC_LIB=LIB)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "checked_runs.py")], env=env,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "checked runs ok" in r.stdout
