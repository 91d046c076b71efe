"""Parity of the HIP adjoint (through the C-ABI) with the FP64 oracle adjoint.

The oracle adjoint is pinned to the forward oracle by test_oracle_adjoint
(dot-product and finite-difference tests).  Here the GPU's FP32 adjoint step,
objective seeds and whole-run gradients (checkpoint-recompute) are compared
with it on the same states.  Tolerances: single adjoint steps and seeds are
FP32 evaluations of O(1) sums, checked at 2e-5 (norm-wise) on lam and 1e-4 per
theta component; whole-run gradients accumulate over hundreds of steps and
are checked against the oracle adjoint run along the GPU's own trajectory
(bounds per objective, set by the FP32 storage of lam; see SAME_TRAJ_TOL),
and at 5e-3 against the all-FP64 run, whose forward trajectory differs from
the FP32 one.  The transpose itself is evaluated in FP64 on the device.
"""
import numpy as np
import pytest

import oracle as O
from paper_1806_06943_amd import adjoint as AD
from paper_1806_06943_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return _t


def say(*a):
    print("[gpu-case]", *a, flush=True)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def droplet_instance(nx, ny, walls=0, R=None, g=1e-5, seed=3, tau=(1.0, 0.6)):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:ny, 0:nx]
    R = R if R is not None else max(2.0, min(nx, ny) / 4)
    disc = (xx - nx / 2 + 0.3) ** 2 + (yy - ny / 2 - 0.2) ** 2 <= R * R
    rhoA = np.where(disc, 1.0, 0.03) + 1e-3 * rng.standard_normal((ny, nx))
    rhoB = np.where(disc, 0.03, 1.0) + 1e-3 * rng.standard_normal((ny, nx))
    return dict(nx=nx, ny=ny, rhoA=rhoA, rhoB=rhoB, G_AB=3.0, G1=-7.4, G2=6.4, tau=tau,
                g=((g, 0.0), (g, 0.0)), walls=walls, rho_wall=(0.03, 1.0))


def oparams(d):
    return O.Params(nx=d["nx"], ny=d["ny"], G_AB=d["G_AB"], G1=d["G1"], G2=d["G2"], tau=d["tau"],
                    g=d["g"], walls=d["walls"], rho_wall=d["rho_wall"])


@pytest.mark.parametrize("nx,ny,walls", [(64, 64, 0), (64, 64, 1), (70, 37, 0), (70, 37, 1),
                                         (5, 3, 0), (130, 9, 1)])
def test_adjoint_step_matches_oracle(torch, nx, ny, walls):
    say("adjoint step", nx, ny, walls)
    d = droplet_instance(nx, ny, walls)
    sim = lbm.Sim([d])
    sim.step(20)
    f = sim.populations()
    rng = np.random.default_rng(nx * 100 + ny + walls)
    lam_in = torch.from_numpy(rng.standard_normal((2, 9, ny, nx)).astype(np.float32)).cuda()
    lam_out = torch.empty_like(lam_in)
    grad = torch.zeros(5, dtype=torch.float64, device="cuda")
    sim.adjoint_step(f, lam_in, lam_out, grad)
    torch.cuda.synchronize()
    lo, go = O.adjoint_step(oparams(d), sim.populations_full(), lam_in.cpu().numpy().astype(np.float64))
    el = rel(lam_out.cpu().numpy(), lo)
    eg = np.abs(grad.cpu().numpy() - go) / np.maximum(np.abs(go), 1e-30)
    say("lam err", el, "grad err", eg)
    assert el <= 2e-5, el
    assert eg.max() <= 1e-4, (eg, grad.cpu().numpy(), go)
    sim.close()


@pytest.mark.parametrize("which", ["dp", "Q", "momA", "mom", "massA"])
@pytest.mark.parametrize("walls", [0, 1])
def test_objective_seed_matches_oracle(torch, which, walls):
    say("seed", which, walls)
    d = droplet_instance(64, 48, walls, g=1e-4)
    sim = lbm.Sim([d])
    sim.step(50)
    f = sim.populations()
    lam = torch.empty_like(f)
    J, dth = sim.adjoint_seed(which, f, lam)
    torch.cuda.synchronize()
    Jo, lo, do = O.objective(oparams(d), sim.populations_full(), which)
    say("J", J, Jo)
    assert abs(J - Jo) <= 1e-6 * abs(Jo) + 1e-9, (J, Jo)
    assert rel(lam.cpu().numpy(), lo) <= 2e-5
    for t in range(5):
        assert abs(dth[t] - do[t]) <= 1e-4 * abs(do[t]) + 1e-12, (t, dth, do)
    sim.close()


def full_f(sim, dev):
    """float64 populations from FP32 deviations."""
    w = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1]) / 36.0
    rr = np.asarray(sim.params[0].rho_ref[:])
    return dev.cpu().numpy().astype(np.float64) + w[None, :, None, None] * rr[:, None, None, None]


def oracle_grad_along(p, states, which):
    """FP64 oracle adjoint along a given trajectory states[0..T]."""
    J, lam, g = O.objective(p, states[-1], which)
    g = g.copy()
    for t in range(len(states) - 2, -1, -1):
        lam, gs = O.adjoint_step(p, states[t], lam)
        g += gs
    return J, g, lam


RUN_STEPS, RUN_WINDOW = 400, 100

# Norm-wise bounds on the same trajectory.  lam is stored in FP32, a relative
# rounding of ~6e-8 per step that random-walks over the run; the gradient of
# a nearly conserved quantity is a small remainder of its per-node terms
# (the flow rate's is ~1e-2 of the scale of the momentum-of-A gradient per
# unit lam), which magnifies that floor.  The zero-gradient test measures the
# floor directly.
SAME_TRAJ_TOL = {"dp": 2e-5, "momA": 2e-4, "Q": 1e-3}


@pytest.fixture(scope="module")
def run_case(torch):
    """64 x 64 periodic droplet of radius 20, g_x = 1e-6, 400 steps: the GPU's own
    trajectory (every state, FP32 cast to FP64) and its oracle parameters."""
    d = droplet_instance(64, 64, 0, R=20, g=1e-6)
    sim = lbm.Sim([d])
    states = [sim.populations_full()]
    for _ in range(RUN_STEPS):
        sim.step(1)
        states.append(sim.populations_full())
    sim.close()
    return d, states


@pytest.mark.parametrize("which", ["dp", "Q", "momA"])
def test_run_gradient_matches_oracle_on_the_same_trajectory(torch, run_case, which):
    """Checkpoint-recompute GPU gradient vs the FP64 oracle adjoint run along the
    GPU's own FP32 trajectory: isolates the adjoint arithmetic."""
    say("run gradient, same trajectory", which)
    d, states = run_case
    prob = AD.Problem(d, steps=RUN_STEPS, objective=which, window=RUN_WINDOW)
    J, g, lam0 = prob.value_and_grad()
    assert np.array_equal(full_f(prob.sim, prob.f0), states[0])
    Jo, go, lo = oracle_grad_along(oparams(d), states, which)
    say("J", J, Jo, "grad", g, go, "rel", rel(g, go))
    assert abs(J - Jo) <= 1e-6 * abs(Jo), (J, Jo)
    assert rel(g, go) <= SAME_TRAJ_TOL[which], (g, go)
    assert rel(lam0.cpu().numpy(), lo) <= 1e-4
    prob.close()


@pytest.mark.parametrize("which", ["dp", "Q", "momA"])
def test_run_gradient_matches_fp64_run(torch, which):
    """GPU gradient vs the all-FP64 oracle run (forward and adjoint in FP64): the
    difference also carries the FP32 forward's trajectory error."""
    say("run gradient, FP64 run", which)
    d = droplet_instance(64, 64, 0, R=20, g=1e-6)
    prob = AD.Problem(d, steps=RUN_STEPS, objective=which, window=RUN_WINDOW)
    J, g, lam0 = prob.value_and_grad()
    Jo, go, lo = O.value_and_grad(oparams(d), full_f(prob.sim, prob.f0), RUN_STEPS, which)
    say("J", J, Jo, "grad", g, go, "rel", rel(g, go))
    assert abs(J - Jo) <= 1e-4 * abs(Jo), (J, Jo)
    assert rel(g, go) <= 5e-3, (g, go)
    assert rel(lam0.cpu().numpy(), lo) <= 5e-3
    prob.close()


@pytest.mark.parametrize("nx,ny,walls,R", [(48, 40, 0, 10), (48, 40, 1, 10), (9, 6, 0, None),
                                           (11, 5, 1, None), (130, 9, 1, None)])
def test_run_equals_single_steps(torch, nx, ny, walls, R):
    """A run of adjoint steps forms each step's pending force-transpose addition
    inside the next step's local pass (from the force adjoints of the step
    before); single adjoint steps run the force pass and fold the addition into
    lam at once.  lam(0) must agree bit for bit, the gradient to FP64 rounding
    (the run sums its per-block partials over all steps before the final sum).
    The small lattices stage tiles mostly past their edge or beyond a wall,
    with halos spanning much of a period."""
    say("run vs single steps", nx, ny, walls)
    d = droplet_instance(nx, ny, walls, R=R, g=1e-5)
    n = 30
    prob = AD.Problem(d, steps=n, objective="dp", window=n)
    J, g, lam0 = prob.value_and_grad()
    prob.close()
    sim = lbm.Sim([d])
    states = [sim.populations()]
    for _ in range(n):
        sim.step(1)
        states.append(sim.populations())
    lam = torch.empty_like(states[-1])
    Js, direct = sim.adjoint_seed("dp", states[-1], lam)
    grad = torch.zeros(5, dtype=torch.float64, device="cuda")
    nxt = torch.empty_like(lam)
    for t in range(n - 1, -1, -1):
        sim.adjoint_step(states[t], lam, nxt, grad)
        lam, nxt = nxt, lam
    torch.cuda.synchronize()
    gs = grad.cpu().numpy() + direct
    say("J", J, Js, "grad", g, gs)
    assert J == Js and np.isfinite(J)
    assert torch.isfinite(lam).all() and torch.equal(lam0, lam)
    assert np.abs(g - gs).max() <= 1e-10 * np.abs(gs).max(), (g, gs)
    sim.close()


def test_conserved_objectives_have_zero_gradient(torch):
    say("zero gradients")
    d = droplet_instance(64, 64, 0, R=16, g=0.0)
    scale = None
    for which in ("momA", "mom", "massA"):
        prob = AD.Problem(d, steps=200, objective=which, window=50)
        J, g, _ = prob.value_and_grad()
        prob.close()
        say(which, J, g)
        if which == "momA":
            scale = np.abs(g).max()  # a non-conserved gradient of comparable magnitude
            continue
        assert np.abs(g).max() <= 1e-4 * scale, (which, g, scale)


@pytest.mark.parametrize("which", ["dp", "momA"])
def test_gradient_does_not_depend_on_the_window(torch, which):
    """Windows re-run on a second stream while the adjoint sweeps the next one:
    J and dJ/df(0) must equal those of one window bit for bit (the re-run
    states are deterministic); the parameter gradient to FP64 rounding (each
    window's per-block partial sums are folded into it at the window's end, so
    the order of the FP64 additions depends on the window)."""
    say("windows", which)
    d = droplet_instance(64, 48, 0, R=12, g=1e-5)
    out = []
    for window in (120, 25, 7):
        prob = AD.Problem(d, steps=120, objective=which, window=window)
        J, g, lam0 = prob.value_and_grad()
        out.append((J, g, lam0.cpu().numpy()))
        prob.close()
    for J, g, lam0 in out[1:]:
        assert J == out[0][0]
        assert np.array_equal(lam0, out[0][2])
        assert np.abs(g - out[0][1]).max() <= 1e-12 * np.abs(out[0][1]).max(), (g, out[0][1])


def test_backward_keeps_to_its_own_forward_pass(torch):
    """The forward pass records its last window for the backward pass; a backward
    pass of an earlier forward pass, or a second backward pass of the same one
    after the store was reused, re-runs that window instead: the gradients equal
    those of a plain forward + backward bit for bit."""
    say("stale store")
    d = droplet_instance(48, 48, 0, R=12, g=1e-5)
    # three windows (the last one's store is reused), two, and one window
    # (steps <= window)
    for window in (30, 45, 90):
        prob = AD.Problem(d, steps=90, objective="dp", window=window)
        th = prob.theta()
        th2 = th.copy()
        th2[2] *= 1.01
        J1, g1, l1 = prob.value_and_grad(th)
        _, s1 = prob.forward(th)
        prob.forward(th2)
        for _ in range(2):
            g, lam = prob.backward(s1)
            assert np.array_equal(g, g1) and torch.equal(lam, l1), window
        _, s3 = prob.forward(th)
        for _ in range(2):  # the recorded window, then (three windows) a re-run
            g, lam = prob.backward(s3)
            assert np.array_equal(g, g1) and torch.equal(lam, l1), window
        # an older forward pass's backward pass re-runs its last window into the
        # store that holds the newer pass's: the newer backward pass must not
        # then take that store as its own
        _, g2, l2 = prob.value_and_grad(th2)
        _, sa = prob.forward(th)
        _, sb = prob.forward(th2)
        g, lam = prob.backward(sa)
        assert np.array_equal(g, g1) and torch.equal(lam, l1), window
        g, lam = prob.backward(sb)
        assert np.array_equal(g, g2) and torch.equal(lam, l2), window
        prob.close()


def test_window_chosen_by_memory(torch):
    """window 0: a run whose states fit in device memory is one window, one
    store, nothing re-run; J and lambda(0) equal the windowed run's bitwise,
    the gradient up to the order of the FP64 per-window sums."""
    say("window by memory")
    d = droplet_instance(48, 48, 0, R=12, g=1e-5)
    a = AD.Problem(d, steps=90, objective="dp", window=0)
    assert a.window == 90
    assert a.auto_window(fraction=1e-12) == 1
    J0, g0, l0 = a.value_and_grad()
    assert a._store.shape[0] == 1
    J1, g1, l1 = a.value_and_grad()  # the recorded run again: bitwise the same
    assert J1 == J0 and np.array_equal(g1, g0) and torch.equal(l1, l0)
    b = AD.Problem(d, steps=90, objective="dp", window=30)
    J2, g2, l2 = b.value_and_grad()
    assert J2 == J0 and torch.equal(l2, l0)
    assert np.allclose(g2, g0, rtol=1e-12, atol=0.0), (g0, g2)
    a.close()
    b.close()


def test_autograd_function_and_finite_differences(torch):
    say("autograd")
    d = droplet_instance(48, 48, 0, R=12, g=1e-5)
    prob = AD.Problem(d, steps=100, objective="dp", window=40)
    theta = torch.tensor(prob.theta(), dtype=torch.float64, requires_grad=True)
    J = AD.objective(theta, prob)
    J.backward()
    g = theta.grad.numpy().copy()
    J2, g2, _ = prob.value_and_grad(prob.theta())
    assert abs(float(J) - J2) == 0.0
    assert np.array_equal(g, g2)
    # central differences of the FP32 forward: a sanity check only (FP32 J has ~1e-7
    # relative noise, so h trades truncation against it)
    base = prob.theta()
    for m, h in enumerate([1e-3, 1e-3, 1e-3, 1e-3, 1e-3]):
        e = np.zeros(5)
        e[m] = h
        Jp, _ = prob.forward(base + e)
        Jm, _ = prob.forward(base - e)
        fd = (Jp - Jm) / (2 * h)
        say("fd", lbm.THETA_NAMES[m], fd, g[m])
        assert abs(fd - g[m]) <= 0.05 * abs(g[m]) + 1e-6 * abs(J2), (m, fd, g[m])
    prob.close()


def test_set_params_changes_the_forward_like_a_fresh_context(torch):
    say("set_params")
    d = droplet_instance(64, 32, 1)
    a = lbm.Sim([d])
    th = a.theta() + np.array([0.1, -0.05, 0.2, 0.1, -0.02])
    a.set_theta(th)
    a.step(40)
    d2 = dict(d, G1=th[0], G2=th[1], G_AB=th[2], tau=(th[3], th[4]))
    b = lbm.Sim([d2])
    b.step(40)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    with pytest.raises(lbm.LBMError):
        p = lbm.lbm_params.from_buffer_copy(a.params[0])
        p.nx = 65
        lbm.lbm_set_params(a.ctx, 0, p)
    a.close()
    b.close()
