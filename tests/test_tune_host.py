"""Host logic of the strip-plan tuner: the fitted-height search, with the
library's workgroup count replaced by the count of a uniform plan (strips x
chunks), so it runs without a GPU."""
import types

import pytest

from paper_1806_06943_amd import tune


class FakeSim:
    def __init__(self, nx, ny):
        self.params = [types.SimpleNamespace(nx=nx, ny=ny)]
        self.ctx = object()
        self.plan = None


def install(monkeypatch, sim, strips):
    """apply() records the plan; lbm_get_workgroups() returns strips * ceil(ny / h)."""
    applied = []

    def apply(s, width, height, balance=0):
        assert height >= tune.MIN_HEIGHT, height  # the library rejects smaller heights
        s.plan = (width, height)
        applied.append(height)

    def workgroups(ctx):
        ny = sim.params[0].ny
        return strips * -(-ny // sim.plan[1])

    monkeypatch.setattr(tune, "apply", apply)
    monkeypatch.setattr(tune.lbm, "lbm_get_workgroups", workgroups)
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
