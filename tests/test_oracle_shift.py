"""Pins of the oracle's velocity-shift forcing (the original two-range model).

Sec. II A writes the velocity shift of the original model as an explicit
forcing term, C^SC = [f^eq(rho, u + F tau / rho) - f^eq(rho, u)] / tau, with
component momenta without F/2.  Fixed here:

* moments of C^SC, from the equilibrium's moments (Eq. 2 with the 1/2):
  sum C = 0, sum C e = F, sum C e e = u F + F u + tau F F / rho (the
  tau-dependent term behind the viscosity dependence the paper removes);
* a step equals BGK towards the equilibrium at the shifted velocity
  u' + tau_k F_k / rho_k, u' the tau-weighted mean of the bare momenta;
* a uniform state is a fixed point; mass is conserved; the population
  momentum grows by exactly sum_k g_k M_k per step (the interaction forces
  sum to zero), as with the Guo term.
"""
import numpy as np
import pytest

import oracle as O

E9 = O.E9


@pytest.mark.parametrize("seed", range(5))
def test_shift_term_moments(seed):
    r = np.random.default_rng(seed)
    tau = 0.55 + 2 * r.random()
    rho = 0.05 + r.random()
    ux, uy, Fx, Fy = 0.05 * r.standard_normal(4)
    C = O.shift(tau, rho, ux, uy, Fx, Fy)
    ex, ey = E9[:, 0], E9[:, 1]
    assert abs(C.sum()) < 1e-15
    assert abs((C * ex).sum() - Fx) < 1e-15 and abs((C * ey).sum() - Fy) < 1e-15
    want = {
        "xx": 2 * ux * Fx + tau * Fx * Fx / rho,
        "yy": 2 * uy * Fy + tau * Fy * Fy / rho,
        "xy": ux * Fy + Fx * uy + tau * Fx * Fy / rho,
    }
    got = {"xx": (C * ex * ex).sum(), "yy": (C * ey * ey).sum(), "xy": (C * ex * ey).sum()}
    for k in want:
        assert abs(got[k] - want[k]) < 1e-14, (k, got[k], want[k])


def _state(p, seed, steps=3):
    r = np.random.default_rng(seed)
    rhoA = 0.5 + 0.3 * r.random((p.ny, p.nx))
    rhoB = 1.0 - rhoA + 0.05 * r.random((p.ny, p.nx))
    return O.run(p, O.init(p, rhoA, rhoB), steps)


@pytest.mark.parametrize("walls", [0, 1])
def test_step_is_bgk_towards_the_shifted_equilibrium(walls):
    p = O.Params(nx=9, ny=7, G_AB=3.0, G1=-7.4, G2=6.4, tau=(0.8, 1.7), forcing=1, walls=walls,
                 rho_wall=(0.2, 0.9), g=((1e-3, 0.0), (2e-4, -1e-4)))
    f = _state(p, 4)
    rho = O.density(p, f)
    F = O.forces(p, rho)
    m = np.einsum("kiyx,id->kdyx", f, E9.astype(float))  # bare momenta [k][d]
    tau = np.array(p.tau)
    D = (rho / tau[:, None, None]).sum(axis=0)
    up = (m / tau[:, None, None, None]).sum(axis=0) / D  # [d][y][x]
    fstar = np.zeros_like(f)
    for k in range(2):
        for y in range(p.ny):
            for x in range(p.nx):
                us = up[:, y, x] + tau[k] * F[k, :, y, x] / rho[k, y, x]
                eq = O.feq(rho[k, y, x], us[0], us[1])
                fstar[k, :, y, x] = f[k, :, y, x] - (f[k, :, y, x] - eq) / tau[k]
    # stream by hand (push, bounce-back across walls)
    want = np.zeros_like(f)
    for k in range(2):
        for i in range(9):
            for y in range(p.ny):
                for x in range(p.nx):
                    yd = y + E9[i, 1]
                    if walls and (yd < 0 or yd >= p.ny):
                        want[k, [0, 3, 4, 1, 2, 7, 8, 5, 6][i], y, x] = fstar[k, i, y, x]
                    else:
                        want[k, i, yd % p.ny, (x + E9[i, 0]) % p.nx] = fstar[k, i, y, x]
    got = O.step(p, f)
    assert np.abs(got - want).max() < 1e-14


def test_uniform_state_is_fixed_point_and_mass_momentum():
    p = O.Params(nx=8, ny=6, G_AB=3.0, G1=-7.4, G2=6.4, tau=(0.7, 1.3), forcing=1)
    f = O.init(p, np.full((6, 8), 0.6), np.full((6, 8), 0.4))
    assert np.abs(O.run(p, f, 5) - f).max() < 1e-15
    g = ((2e-4, 0.0), (1e-4, -3e-4))
    p = O.Params(nx=12, ny=10, G_AB=3.0, G1=-7.4, G2=6.4, tau=(0.7, 1.3), forcing=1, g=g)
    f = _state(p, 9)
    M0 = O.masses(f)
    P0 = O.raw_momentum(f)
    f1 = O.run(p, f, 25)
    assert np.allclose(O.masses(f1), M0, rtol=1e-13, atol=0)
    gg = np.asarray(g)
    dP = 25 * (gg * M0[:, None]).sum(axis=0)
    assert np.allclose(O.raw_momentum(f1) - P0, dP, rtol=1e-10, atol=1e-13)


def test_schemes_differ_only_through_the_force():
    """With no force anywhere (G = 0, g = 0) the two schemes are the same BGK step."""
    p0 = O.Params(nx=10, ny=8, G_AB=0.0, G1=0.0, G2=0.0, tau=(0.8, 1.6), forcing=0)
    p1 = O.Params(nx=10, ny=8, G_AB=0.0, G1=0.0, G2=0.0, tau=(0.8, 1.6), forcing=1)
    f = _state(p0, 2)
    assert np.abs(O.run(p0, f, 7) - O.run(p1, f, 7)).max() < 1e-15


def _slab(p, steps, f=None):
    nx, ny = p.nx, p.ny
    if f is None:
        x = np.arange(nx)
        slab = (x >= nx // 4) & (x < 3 * nx // 4)
        rA = np.repeat(np.where(slab, 1.0, 0.03)[None, :], ny, axis=0)
        rB = np.repeat(np.where(slab, 0.03, 1.0)[None, :], ny, axis=0)
        f = O.init(p, rA, rB)
    nthr = O.threads()
    O.set_threads(1)  # a two-row slab: no fork and join per step
    try:
        return O.run(p, f, steps)
    finally:
        O.set_threads(nthr)


def test_original_model_at_the_emulsion_couplings():
    """Why the original model's numbers of Sec. III C (gamma = 0.043 at M = 1) are
    not reproduced by the shift of Eq. 4 at the emulsion couplings (3.0, -7.4, 6.4):
    on a relaxed flat interface the Eq. 9 repulsion per unit density of the
    minority component is not small (|F_k / rho_k| > 0.4), so at tau = 0.8 (the
    viscosity of Figs. 5-6) the shifted equilibrium drives the minority density
    below zero, and at tau = 1 the shift is stable but changes the coexistence
    (minority density 0.004 against 0.019) and gamma (about 0.16; Sigma f e e and
    the exact plane-flux balance agree on it, see test_oracle_pressure_pins)."""
    G_AB, G1, G2 = 3.0, -7.4, 6.4
    kw = dict(nx=96, ny=2, G_AB=G_AB, G1=G1, G2=G2)
    guo = O.Params(tau=(1.0, 1.0), **kw)
    f = _slab(guo, 20000)
    rho = O.density(guo, f)
    F = O.forces(guo, rho)
    assert np.abs(F[:, 0] / rho).max() > 0.4
    g_guo = O.line_tension(O.pressure(guo, f)) / 2
    assert abs(g_guo - 0.043) < 0.002  # the present model: Sec. III D's value
    # tau = 0.8: bounded, but the minority density goes negative
    p8 = O.Params(tau=(0.8, 0.8), forcing=1, **kw)
    f8 = _slab(p8, 5000, f)
    r8 = O.density(p8, f8)
    assert np.isfinite(f8).all() and r8.min() < -0.005
    # tau = 1: stable, different coexistence and a surface tension near 0.16
    p1 = O.Params(tau=(1.0, 1.0), forcing=1, **kw)
    f1 = _slab(p1, 20000, f)
    r1 = O.density(p1, f1)
    assert 0.0 < r1.min() < 0.006 and rho.min() > 0.015
    g1 = O.line_tension(O.pressure(guo, f1)) / 2  # kinetic tensor sum f e e
    assert 0.15 < g1 < 0.17, g1
