import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU runs of the oracle (deselect with -m 'not slow')")


def read_golden(name: str = "paper_values.txt") -> dict:
    """key = value lines; values may be fractions 'a/b' or decimals."""
    from fractions import Fraction
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            out[k] = Fraction(v)
    return out


@pytest.fixture(scope="session")
def golden():
    return read_golden()
