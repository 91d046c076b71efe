"""Host logic of the strip-plan tuner: the fitted-height search, with the
library's host planner replaced by the count of a uniform plan (strips x
chunks), so the search itself is checked against a brute force."""
import types

import pytest

from paper_1806_06943_amd import tune


class FakeSim:
    def __init__(self, nx, ny):
        self.params = [types.SimpleNamespace(nx=nx, ny=ny)]
        self.ctx = object()
        self.plan = None


def install(monkeypatch, sim, strips):
    """lbm_plan_workgroups() records the height and returns strips * ceil(ny / h)."""
    applied = []

    def plan(params, width, height, wgs=0, full_rows=0):
        assert tune.MIN_HEIGHT <= height <= tune.MAX_HEIGHT, height  # the library's range
        applied.append(height)
        ny = params[0].ny
        n = strips * -(-ny // height)
        return n, n

    monkeypatch.setattr(tune.lbm, "lbm_plan_workgroups", plan)
    return applied


@pytest.mark.parametrize("ny,strips,ncu", [(2048, 5, 256), (2048, 9, 256), (2048, 34, 256),
                                            (512, 3, 256), (40, 10, 256), (2048, 17, 80)])
def test_fitted_heights_are_the_smallest_within_each_multiple(monkeypatch, ny, strips, ncu):
    sim = FakeSim(2048, ny)
    install(monkeypatch, sim, strips)
    hs = tune.fitted_heights(sim, 240, ncu)

    def wg(h):
        return strips * -(-ny // h)

    want = set()
    for k in range(1, tune.FIT_KMAX + 1):
        ok = [h for h in range(tune.MIN_HEIGHT, max(ny, tune.MIN_HEIGHT) + 1) if wg(h) <= k * ncu]
        if ok:
            want.add(min(ok))
    assert hs == sorted(want)


def test_no_height_below_the_library_minimum_is_tried(monkeypatch):
    # one-wave strips on a wide lattice: k * ncu workgroups need heights below 4
    sim = FakeSim(2048, 2048)
    applied = install(monkeypatch, sim, 34)
    hs = tune.fitted_heights(sim, 58, 256)
    assert min(applied) >= tune.MIN_HEIGHT and all(h >= tune.MIN_HEIGHT for h in hs)


def test_fitted_heights_of_a_real_plan_stay_in_range():
    """With the library's own host planner: the accepted 64 x 466033 lattice (more
    rows than one chunk may hold) gets heights within the range of lbm_set_tiling."""
    from paper_1806_06943_amd import lbm
    p = lbm.make_params(nx=64, ny=466033, G_AB=3.0, G1=-7.4, G2=6.4, tau=(1.0, 0.6), walls=1)
    sim = FakeSim(64, 466033)
    sim.params = [p]
    for fr in (0, 1):
        hs = tune.fitted_heights(sim, 58, 256, full_rows=fr)
        assert hs and all(tune.MIN_HEIGHT <= h <= tune.MAX_HEIGHT for h in hs)
