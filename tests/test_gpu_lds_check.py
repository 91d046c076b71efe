"""The checked build of the library (compiled with LBM_CHECK_LDS) counts every
out-of-range index of the fused step's LDS ring and edge arrays instead of
using it.  Strip plans of 1 to 8 wavefronts (uniform and balanced), lattices
narrower than a strip, one-column and one-row tori, walls, and full-row
plans (single and mixed widths, a recorded window) must count none.  Runs in a
child process because a process loads one build of the library."""
import os
import subprocess
import sys

import pytest

from paper_1806_06943_amd import build as HB

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_no_lds_index_leaves_its_array():
    if not os.path.exists(HB.CHECKED):
        pytest.fail("the checked build is missing: run __graft_entry__.build()")
    env = dict(os.environ, LBM_HIP_SO=HB.CHECKED)
    print("[gpu-case] LDS checks in a child process", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "lds_check_cases.py")],
                       env=env, capture_output=True, text=True, timeout=600)
    log = r.stdout + r.stderr
    assert r.returncode == 0, log[-3000:]
    last = [l for l in log.splitlines() if l.startswith("LDS_VIOLATIONS")]
    assert last and last[-1] == "LDS_VIOLATIONS 0", log[-3000:]
