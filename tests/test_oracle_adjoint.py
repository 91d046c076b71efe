"""Pins of the FP64 oracle adjoint against the forward oracle.

The adjoint of a step is, by definition, the transpose of the step's
derivative.  The forward oracle is pinned to the paper by test_oracle_pins;
here its central differences fix the adjoint:

* dot-product test: <lam_next, (Phi(f + h df) - Phi(f - h df)) / 2h> equals
  <(dPhi/df)^T lam_next, df>, periodic and walled, with body force;
* parameter derivative of one step against central differences in theta;
* objective seeds against central differences of the objective;
* whole-run gradients (30 steps, a droplet) against central differences;
* conserved quantities: the gradients of the mass of A and of the total
  population momentum vanish, because mass is conserved and the interaction
  forces of Eqs. 8, 9 sum to zero over a torus (pairwise antisymmetry).
"""
import numpy as np
import pytest

import oracle as O

TH = O.THETA_NAMES


def rand_state(p, rng, steps=3):
    rhoA = 0.5 + 0.3 * rng.random((p.ny, p.nx))
    rhoB = 1.0 - rhoA + 0.05 * rng.random((p.ny, p.nx))
    f = O.run(p, O.init(p, rhoA, rhoB), steps)
    w = np.array(O.tables()[3])
    return f + 0.01 * rng.standard_normal(f.shape) * w[None, :, None, None]


def params(walls, nx=12, ny=10):
    return O.Params(nx=nx, ny=ny, G_AB=3.0, G1=-7.4, G2=6.4, tau=(0.8, 1.3),
                    g=((1e-3, 2e-4), (5e-4, -3e-4)), walls=walls, rho_wall=(0.2, 0.9))


@pytest.mark.parametrize("walls", [0, 1])
def test_dot_product_one_step(walls):
    rng = np.random.default_rng(10 + walls)
    p = params(walls)
    f = rand_state(p, rng)
    lam_next = rng.standard_normal(f.shape)
    df = rng.standard_normal(f.shape)
    lam, _ = O.adjoint_step(p, f, lam_next)
    h = 1e-6
    tang = (O.step(p, f + h * df) - O.step(p, f - h * df)) / (2 * h)
    a = (lam_next * tang).sum()
    b = (lam * df).sum()
    assert abs(a - b) <= 1e-9 * abs(a), (a, b)


@pytest.mark.parametrize("walls", [0, 1])
def test_parameter_derivative_one_step(walls):
    rng = np.random.default_rng(20 + walls)
    p = params(walls)
    f = rand_state(p, rng)
    lam_next = rng.standard_normal(f.shape)
    _, g = O.adjoint_step(p, f, lam_next)
    th = O.theta_of(p)
    for m in range(5):
        e = np.zeros(5)
        e[m] = 1e-6
        tp = (O.step(O.with_theta(p, th + e), f) - O.step(O.with_theta(p, th - e), f)) / 2e-6
        a = (lam_next * tp).sum()
        assert abs(a - g[m]) <= 1e-6 * abs(a), (TH[m], a, g[m])


def droplet_problem(nx=24, ny=20, seed=1, g=1e-4):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:ny, 0:nx]
    disc = (xx - 11.3) ** 2 + (yy - 9.6) ** 2 <= 36
    rhoA = np.where(disc, 1.0, 0.03) + 1e-3 * rng.standard_normal((ny, nx))
    rhoB = np.where(disc, 0.03, 1.0) + 1e-3 * rng.standard_normal((ny, nx))
    p = O.Params(nx=nx, ny=ny, G_AB=3.0, G1=-7.4, G2=6.4, tau=(1.0, 0.6), g=((g, 0), (g, 0)))
    return p, O.init(p, rhoA, rhoB)


@pytest.mark.parametrize("which", ["dp", "Q", "momA", "mom", "massA"])
def test_objective_seed(which):
    p, f0 = droplet_problem()
    f = O.run(p, f0, 5)
    J, lam, _ = O.objective(p, f, which)
    rng = np.random.default_rng(5)
    df = 1e-2 * rng.standard_normal(f.shape)
    h = 1e-6
    a = (O.objective(p, f + h * df, which)[0] - O.objective(p, f - h * df, which)[0]) / (2 * h)
    b = (lam * df).sum()
    assert abs(a - b) <= 1e-6 * abs(b), (a, b)


@pytest.mark.parametrize("which", ["dp", "Q", "momA"])
def test_run_gradient_matches_central_differences(which):
    p, f0 = droplet_problem()
    steps = 30
    J, g, lam0 = O.value_and_grad(p, f0, steps, which)
    th = O.theta_of(p)
    for m in range(5):
        e = np.zeros(5)
        e[m] = 1e-5
        fd = (O.objective_after(O.with_theta(p, th + e), f0, steps, which)
              - O.objective_after(O.with_theta(p, th - e), f0, steps, which)) / 2e-5
        assert abs(fd - g[m]) <= 1e-5 * abs(g[m]) + 1e-12, (which, TH[m], fd, g[m])
    # gradient with respect to the initial state
    rng = np.random.default_rng(7)
    df = 1e-3 * rng.standard_normal(f0.shape)
    h = 1e-5
    fd = (O.objective_after(p, f0 + h * df, steps, which)
          - O.objective_after(p, f0 - h * df, steps, which)) / (2 * h)
    assert abs(fd - (lam0 * df).sum()) <= 1e-6 * abs(fd), (fd, (lam0 * df).sum())


# (walls exchange momentum with the fluid, so the momentum case is periodic only)
@pytest.mark.parametrize("which,walls", [("mom", 0), ("massA", 0), ("massA", 1)])
def test_conserved_quantities_have_zero_parameter_gradient(which, walls):
    p, f0 = droplet_problem()
    if walls:
        p = O.Params(**{**p.__dict__, "walls": 1, "rho_wall": (0.03, 1.0)})
    steps = 20
    J, g, lam0 = O.value_and_grad(p, f0, steps, which)
    assert np.abs(g).max() <= 1e-12 * max(1.0, abs(J)), g
    # d J(T) / d f(0): the mass of A is conserved; the momentum grows by
    # sum_k g_k M_k per step, so d P_x(T) / d f_{k,i} = e_{i,x} + T g_{k,x}
    _, lamT, _ = O.objective(p, f0, which)
    want = lamT.copy()
    if which == "mom":
        gx = np.asarray(p.g, dtype=np.float64).reshape(2, 2)[:, 0]
        want += steps * gx[:, None, None, None]
    assert np.allclose(lam0, want, rtol=0, atol=1e-12)
