"""Checkpoint and resume: a state exported with lbm_get_populations after n steps
and imported into a fresh context with lbm_set_populations continues exactly as
the uninterrupted run, bit for bit (the populations are the whole state: the
step derives every density it uses from them), through single launches and
replayed graphs, for one instance and for one instance of a batch, and under a
different strip plan in the resumed context."""
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


CASES = {
    "droplet": lambda: [W.droplet(nx=96, ny=80, radius=18, couplings=W.COUPLINGS_PAPER,
                                  tau=(1.0, 0.6))],
    "walled": lambda: [W.emulsion(nx=200, ny=72, ndrop=3, radius=9, tau_ratio=2.0, gx=1e-5)],
    "batch": lambda: [W.droplet(nx=64, ny=64, radius=12, couplings=W.COUPLINGS_PAPER,
                                tau=(1.6, 1.0), sub=3),
                      W.emulsion(nx=130, ny=40, ndrop=2, radius=7, gx=1e-5)],
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("n,m", [(37, 5), (137, 200)])
def test_resume_is_bitwise_equal(torch, case, n, m):
    ws = CASES[case]()
    insts = [lbm.workload_instance(w) for w in ws]
    say("resume", case, n, m)
    a = lbm.Sim(insts)
    a.step(n)
    ck = [a.populations(i).clone() for i in range(len(ws))]
    a.step(m)
    want = [a.populations(i).cpu().numpy() for i in range(len(ws))]
    obs_a, _ = a.observables()
    a.close()
    b = lbm.Sim(insts)
    lbm.lbm_set_strip_width(b.ctx, 112)  # another plan: results do not depend on it
    lbm.lbm_set_tiling(b.ctx, 7)
    for i in range(len(ws)):
        b.set_populations(ck[i], i)
    assert b.steps_done == 0
    b.step(m)
    for i in range(len(ws)):
        assert np.array_equal(b.populations(i).cpu().numpy(), want[i]), (case, i)
    obs_b, _ = b.observables()
    for i in range(len(ws)):
        assert obs_b[i]["mass"] == obs_a[i]["mass"] and obs_b[i]["mom_raw"] == obs_a[i]["mom_raw"]
    b.close()
