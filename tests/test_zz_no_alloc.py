"""lbm_observables_noalloc (the entry point for callers that cannot allocate)
against lbm_observables, through the C-ABI: the same kernels over a static
device scratch array instead of the workspace, so every field must be equal
bit for bit.  Two calls in a row, the second on a smaller input (fewer rows
and instances than the first left in the shared array), then a context too
large for the array, which must be refused."""
import ctypes
import math

import numpy as np
import pytest

from paper_1806_06943_amd import lbm
from paper_1806_06943_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return _t


def say(*a):
    print("[gpu-case]", *a, flush=True)


def same(a, b):
    if isinstance(a, list):
        return len(a) == len(b) and all(same(x, y) for x, y in zip(a, b))
    if isinstance(a, float) and math.isnan(a):
        return isinstance(b, float) and math.isnan(b)
    return a == b


def compare(sim):
    rc0, ref, _ = lbm.lbm_observables(sim.ctx, sim.n_inst, None)
    out = (lbm.lbm_obs * sim.n_inst)()
    rc = lbm.lib().lbm_observables_noalloc(sim.ctx, out)
    assert rc == rc0 == lbm.LBM_OK, (rc, rc0)
    got = [o.as_dict() for o in out]
    for i, (g, r) in enumerate(zip(got, ref)):
        for k in r:
            assert same(g[k], r[k]), (i, k, g[k], r[k])
    return got


def test_noalloc_observables_equal_the_workspace_ones(torch):
    # first call: three instances (two droplets and a walled channel), 224 rows
    ws = [W.droplet(nx=96, ny=96, radius=20, couplings=W.COUPLINGS_PAPER, tau=(1.0, 0.6)),
          W.droplet(nx=64, ny=48, radius=10, couplings=W.COUPLINGS_PAPER, tau=(1.6, 1.0), sub=1),
          W.emulsion(nx=128, ny=80, ndrop=3, radius=10, gx=1e-5)]
    insts = [lbm.workload_instance(w) for w in ws[:2]]
    e = lbm.workload_instance(ws[2])
    insts.append(e)
    say("noalloc call 1: 3 instances")
    # instances of one context may differ in walls and body force
    sim = lbm.Sim(insts)
    sim.step(150)
    big = compare(sim)
    assert all(o["finite"] for o in big)
    sim.close()
    # second call: one smaller instance, fewer rows and results than the first
    say("noalloc call 2: 1 smaller instance")
    w = W.droplet(nx=40, ny=40, radius=9, couplings=W.COUPLINGS_PAPER, tau=(1.0, 1.0), sub=2)
    sim = lbm.Sim([lbm.workload_instance(w)])
    sim.step(60)
    small = compare(sim)
    assert small[0]["mass"] != big[0]["mass"]
    sim.close()


def test_noalloc_refuses_contexts_beyond_its_scratch(torch):
    # 12 doubles per row: 50000 rows need more than the 2^19 doubles of scratch
    say("noalloc refusal")
    ny = 50000
    rA = np.full((ny, 16), 0.5)
    inst = dict(nx=16, ny=ny, rhoA=rA, rhoB=1.0 - rA, G_AB=0.405, G1=-9.0, G2=8.1,
                tau=(1.0, 0.6))
    sim = lbm.Sim([inst])
    out = (lbm.lbm_obs * 1)()
    rc = lbm.lib().lbm_observables_noalloc(sim.ctx, out)
    assert rc == lbm.LBM_EINVAL
    assert b"scratch" in lbm.lib().lbm_last_error(sim.ctx)
    # the workspace path still serves it
    rc0, ref, _ = lbm.lbm_observables(sim.ctx, 1, None)
    assert rc0 == lbm.LBM_OK and ref[0]["finite"]
    sim.close()
