"""Two steps per launch (lbm_set_two_step, k_fused_step2) against the single
step: every node goes through the operations of two single steps in the same
order, so the states must be equal bit for bit, for periodic and walled
lattices, narrow and one-row lattices, mixed sizes in one context, strip
widths and heights down to the smallest, balanced plans, odd step counts
(the last step alone), graph replays and both forcing schemes."""
import numpy as np
import pytest

from paper_1806_06943_amd import lbm, tune
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


def instances(spec, forcing=0):
    out = []
    for j, (nx, ny, walls) in enumerate(spec):
        r = np.random.default_rng(2000 + 31 * j + nx + 7 * ny)
        yy, xx = np.mgrid[0:ny, 0:nx]
        disc = (xx - nx / 3) ** 2 + (yy - ny / 2) ** 2 <= (min(nx, ny) / 3) ** 2
        rA = np.where(disc, 1.0, 0.03) + r.uniform(-1e-3, 1e-3, (ny, nx))
        rB = np.where(disc, 0.03, 1.0) + r.uniform(-1e-3, 1e-3, (ny, nx))
        out.append(dict(nx=nx, ny=ny, rhoA=rA, rhoB=rB, G_AB=3.0, G1=-7.4, G2=6.4,
                        tau=(1.0, 1.0) if forcing else (1.0, 0.7), walls=walls,
                        rho_wall=(0.03, 1.0), g=((2e-5, 1e-6), (2e-5, 1e-6)), forcing=forcing))
    return out


CASES = {
    "40x33": [(40, 33, 0)],
    "100x57w": [(100, 57, 1)],
    "256x48": [(256, 48, 0)],
    "53x1": [(53, 1, 0)],
    "17x70w": [(17, 70, 1)],
    "mixed": [(64, 64, 0), (130, 40, 1), (52, 30, 0), (200, 25, 1), (16, 9, 1)],
}


def states(sim, n):
    """The instances' populations as raw bits, every NaN as one canonical
    pattern.  A tiny walled lattice of the mixed case goes unstable under the
    velocity shift: where its NaNs are compared, but not their sign and
    payload, which IEEE 754 leaves to the implementation for an operation on
    NaNs and which follow the operand order the compiler picks for a
    commutative instruction."""
    out = []
    for i in range(n):
        f = sim.populations(i).cpu().numpy()
        b = f.view(np.uint32).copy()
        b[np.isnan(f)] = 0x7FC00000
        out.append(b)
    return out


@pytest.mark.parametrize("case", sorted(CASES))
def test_two_step_equals_single_steps(torch, case):
    say("two steps", case)
    for forcing in (0, 1):
        insts = instances(CASES[case], forcing)
        n = len(insts)
        ref = {}
        for steps in (23, 32):
            sim = lbm.Sim(insts)
            sim.step(steps)
            ref[steps] = states(sim, n)
            sim.close()
        for width, h, bal in ((52, 0, 0), (52, 2, 0), (48, 3, 0), (20, 7, 0), (16, 65535, 0),
                              (52, 0, 2)):
            for steps in (23, 32):
                sim = lbm.Sim(insts)
                tune.apply(sim, width, h or 16, bal, 0, 1)
                assert lbm.lbm_get_two_step(sim.ctx) == 1
                sim.step(steps)  # 32: two graph replays of 8 launches; 23: 11 launches + 1 step
                f = states(sim, n)
                assert lbm.lbm_steps_done(sim.ctx) == steps
                sim.close()
                for i in range(n):
                    assert np.array_equal(f[i], ref[steps][i]), (case, forcing, width, h, bal, steps, i)


def test_two_step_long_run_and_mode_switches(torch):
    """200 steps of a 256^2 spinodal, switching between single and two-step
    launches (and strip plans) on the way, equal the single step's states."""
    w = W.spinodal(nx=256, ny=256)
    a = lbm.Sim([lbm.workload_instance(w)])
    a.step(200)
    ref = a.populations().cpu().numpy()
    a.close()
    b = lbm.Sim([lbm.workload_instance(w)])
    tune.apply(b, 52, 40, 0, 0, 1)
    b.step(61)
    tune.apply(b, 58, 16)
    b.step(13)
    tune.apply(b, 48, 0, 3, 0, 1)
    b.step(126)
    assert np.array_equal(b.populations().cpu().numpy(), ref) and np.isfinite(ref).all()
    b.close()


def test_two_step_droplet_against_the_oracle(torch):
    """The two-step path against the FP64 oracle directly: the 64 x 64 droplet
    with its literal couplings after 200 steps (odd launches count: 100 two-step
    launches), rho and u within 1e-5 norm-wise like the single step."""
    import oracle as O
    w = W.droplet(nx=64, ny=64, radius=12, couplings=W.COUPLINGS_LITERAL, tau=(1.0, 0.6))
    sim = lbm.Sim([lbm.workload_instance(w)])
    tune.apply(sim, 52, 16, 0, 0, 1)
    sim.step(200)
    rho, u = sim.fields()
    p = O.Params(nx=w.nx, ny=w.ny, G_AB=w.G_AB, G1=w.G1, G2=w.G2, tau=w.tau)
    fl = O.fields(p, O.run(p, O.init(p, w.rhoA, w.rhoB), 200))
    rho, u = rho.cpu().numpy(), u.cpu().numpy()
    err_rho = np.linalg.norm(rho - fl["rho"]) / np.linalg.norm(fl["rho"])
    err_u = np.linalg.norm(u - fl["u"]) / np.linalg.norm(fl["u"])
    say("two-step droplet vs oracle", err_rho, err_u)
    assert err_rho < 1e-5 and err_u < 1e-5, (err_rho, err_u)
    sim.close()


def test_two_step_refused_plans_and_profile(torch):
    sim = lbm.Sim(instances([(128, 40, 0)]))
    lbm.lbm_set_strip_width(sim.ctx, 58)
    with pytest.raises(lbm.LBMError):
        lbm.lbm_set_two_step(sim.ctx, 1)
    assert lbm.lbm_get_two_step(sim.ctx) == 0
    lbm.lbm_set_strip_width(sim.ctx, 52)
    lbm.lbm_set_two_step(sim.ctx, 1)
    for bad in (lambda: lbm.lbm_set_strip_width(sim.ctx, 58),
                lambda: lbm.lbm_set_strip_width(sim.ctx, 122),
                lambda: lbm.lbm_set_full_rows(sim.ctx, 1)):
        with pytest.raises(lbm.LBMError):
            bad()
    assert lbm.lbm_get_two_step(sim.ctx) == 1 and lbm.lbm_get_strip_width(sim.ctx) == 52
    for bad in (53, 116):
        with pytest.raises(lbm.LBMError):
            lbm.lbm_set_strip_width(sim.ctx, bad)
    prof = dict(lbm.lbm_profile_step(sim.ctx, 5))
    assert set(prof) == {"k_fused_step2"} and prof["k_fused_step2"] > 0.0
    lbm.lbm_set_two_step(sim.ctx, 0)
    assert set(dict(lbm.lbm_profile_step(sim.ctx, 5))) == {"k_fused_step"}
    sim.close()
