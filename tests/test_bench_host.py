"""Host-side checks of bench.py's counter tables and roofline arithmetic (no GPU)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_counter_tables_cover_the_same_sources_and_plans():
    assert bench.MEASURED_VALU["src_sha256_16"] == bench.MEASURED_TRAFFIC["src_sha256_16"]
    assert set(bench.MEASURED_VALU["plans"]) == set(bench.MEASURED_TRAFFIC["plans"])
    for key, insts in bench.MEASURED_VALU["plans"].items():
        assert key[0] in ("spinodal", "batched") and isinstance(insts, int) and insts > 0


def test_valu_issue_peak_from_the_unit_counts():
    # 256 CUs x 4 SIMDs of 16 lanes: a wave64 instruction every 4 cycles at 2.4 GHz
    assert bench.VALU_ISSUE_PEAK == pytest.approx(614.4)
    # one FMA (2 FLOP) per lane of each instruction: the FP32 vector peak without packed math
    assert bench.VALU_ISSUE_PEAK * 64 * 2 / 1000 == pytest.approx(78.6432)


def test_valu_roofline_arithmetic():
    r = bench.valu_roofline(80161640, 0.16346)
    assert r["bound"] == "alu" and r["unit"] == "G wave64 VALU instructions/s"
    assert r["achieved"] == pytest.approx(80161640 / 0.16346e-3 / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / 614.4, abs=1e-4)
    assert bench.valu_roofline(None, 0.1) is None
