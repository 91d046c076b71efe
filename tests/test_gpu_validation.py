"""The paper's validations run on the HIP path at the paper's sizes.

* Two-component Poiseuille flow (Sec. III A, Eq. 19): 10 x 160 channel,
  half-way bounce-back walls, b = 2a = 80, centreline velocity 0.05, viscosity
  ratios M = mu_B / mu_A in {1/50, 1, 50}, for the paper's three couplings
  (G_A1 = -6 and -8 with G_A2 = -1 - G_A1, and the reference G_A1 = G_A2 = 0).
  The steady profile must follow Eq. 19 away from the diffuse interface.
* Spurious currents (Appendix): the maximum velocity around a steady droplet
  of radius 20 with the couplings of Sec. III D grows as M falls and shrinks
  as G_A1 grows (droplet at tau_A = 1, the matrix's tau_B setting M; the
  figure's values are not in the text, so the trends are what is checked).
  Below M = 1/10 this droplet diverges at these couplings, in the FP64
  oracle as well.

* Pressure tensor (Sec. II B): the library's tensor and line tension against
  the oracle's; flat-interface gamma = 0.04 independent of M within 1.2 %
  (Sec. III C); disjoining pressure (Eqs. 16-18) with the shapes of Fig. 3a.
* Droplet collisions (Sec. III C, Figs. 5-6): two equal droplets of A in B
  meeting head-on at Ca ~ 0.3 and We ~ 15 bounce back under the present model
  at M = 1 and M = 3 (the film of B between them survives); the single-range
  model coalesces in the same collision; the original model bounces at M = 1.
* Emulsion viscosity (Sec. III D, Eq. 20): a walled 220 x 220 channel at
  F_b-bar = 37 and M = 1 with 5 x 5 droplets; the relative viscosity
  Q(0) / Q(Phi) rises with Phi and stays within 10 % of the paper's fit
  (K = 1, [eta] = 0.88) up to Phi = 0.37, and the droplet-free channel carries
  the Poiseuille flow rate.

Viscosities in Eq. 19 are the bulk-phase mixture viscosities sum_k rho_k nu_k,
as in the oracle's pin of the same flow.
"""
import numpy as np
import pytest

import oracle as O
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


def taus_for(M):
    """tau_A, tau_B for mu_B / mu_A = M with the larger one at 1."""
    if M <= 1:
        return 1.0, 0.5 + M * 0.5
    return 0.5 + 0.5 / M, 1.0


POIS_TOL = {  # max |u - u_Eq19| / u0 away from the interface
    (-6.0, 1.0): 0.03, (-6.0, 50.0): 0.03, (-6.0, 1 / 50): 0.06,
    (-8.0, 1.0): 0.03, (-8.0, 50.0): 0.03, (-8.0, 1 / 50): 0.06,
    (0.0, 1.0): 0.03, (0.0, 50.0): 0.03, (0.0, 1 / 50): 0.06,
}


@pytest.mark.parametrize("G1,M", sorted(POIS_TOL))
def test_poiseuille_profile_on_gpu(torch, G1, M):
    say("poiseuille", G1, M)
    nx, ny = 10, 160
    b, a = ny / 2, ny / 4
    u0 = 0.05
    G2 = 0.0 if G1 == 0.0 else -1.0 - G1
    tauA, tauB = taus_for(M)
    nu = ((tauA - 0.5) / 3, (tauB - 0.5) / 3)
    y = np.abs(np.arange(ny) - (ny - 1) / 2.0)
    core = y < a
    rA = np.repeat(np.where(core, 0.03, 1.0)[:, None], nx, axis=1)
    rB = np.repeat(np.where(core, 1.0, 0.03)[:, None], nx, axis=1)
    inst = dict(nx=nx, ny=ny, rhoA=rA, rhoB=rB, G_AB=3.0, G1=G1, G2=G2, tau=(tauA, tauB),
                walls=1, rho_wall=(1.0, 0.03))
    sim = lbm.Sim([inst])
    sim.step(20000)  # interfaces settle, no flow
    rho, _ = sim.fields()
    rho = rho.cpu().numpy().astype(np.float64)[:, :, 0]
    film, cen = int(ny / 2 + (a + b) / 2), ny // 2
    muA = rho[0, film] * nu[0] + rho[1, film] * nu[1]
    muB = rho[0, cen] * nu[0] + rho[1, cen] * nu[1]
    Fb = u0 / (a * a / (2 * muB) + (b * b - a * a) / (2 * muA))
    ua = np.where(y < a, Fb / (2 * muB) * (a * a - y * y) + Fb / (2 * muA) * (b * b - a * a),
                  Fb / (2 * muA) * (b * b - y * y))
    # start from the settled densities moving with the analytic profile
    f = np.zeros((2, 9, ny, nx))
    for yy in range(ny):
        for k in range(2):
            f[k, :, yy, :] = O.feq(rho[k, yy], ua[yy], 0.0)[:, None]
    p = sim.params[0]
    w = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1]) / 36.0
    dev = f - w[None, :, None, None] * np.asarray(p.rho_ref[:])[:, None, None, None]
    sim.set_populations(torch.from_numpy(dev.astype(np.float32)).cuda())
    gx = Fb / rho.sum(axis=0).mean()
    q = lbm.lbm_params.from_buffer_copy(p)
    q.g[0][0] = q.g[1][0] = gx
    lbm.lbm_set_params(sim.ctx, 0, q)
    sim.step(100000)
    _, u = sim.fields()
    ux = u.cpu().numpy().astype(np.float64)[0].mean(axis=1)
    sim.close()
    far = np.abs(y - a) > 5
    err = np.abs(ux - ua)[far].max() / u0
    say("max error / u0 away from the interface", err)
    assert err < POIS_TOL[(G1, M)], err


def spurious_current(torch, M, G1, steps=30000, n=128, R=20):
    # the droplet keeps tau_A = 1; the matrix's tau_B sets M = mu_B / mu_A
    tauA, tauB = taus_for(M)
    say("droplet M", M, "G_A1", G1, "tau", (tauA, tauB))
    yy, xx = np.mgrid[0:n, 0:n]
    disc = (xx - n / 2 + 0.5) ** 2 + (yy - n / 2 + 0.5) ** 2 <= R * R
    inst = dict(nx=n, ny=n, rhoA=np.where(disc, 1.0, 0.03), rhoB=np.where(disc, 0.03, 1.0),
                G_AB=3.0, G1=G1, G2=-1.0 - G1, tau=(tauA, tauB))
    sim = lbm.Sim([inst])
    sim.step(steps)
    obs, _ = sim.observables()
    sim.close()
    say("u_s", obs[0]["max_speed"])
    return obs[0]["max_speed"]


def test_spurious_currents_follow_the_papers_trends(torch):
    say("spurious currents")
    us = {}
    for M in (1 / 10, 1 / 5, 1.0):
        us[(M, -7.4)] = spurious_current(torch, M, -7.4)
    for G1 in (-8.0, -6.0):
        us[(1.0, G1)] = spurious_current(torch, 1.0, G1)
    for k, v in sorted(us.items()):
        say("M", k[0], "G_A1", k[1], "u_s", v)
    # grows as M falls
    assert us[(1 / 10, -7.4)] > us[(1 / 5, -7.4)] > us[(1.0, -7.4)]
    # shrinks as G_A1 grows
    assert us[(1.0, -8.0)] > us[(1.0, -7.4)] > us[(1.0, -6.0)]


# ---------------------------------------------------------------- pressure tensor
def slab_instance(nx, ny, film, G1, G2, tau=(1.0, 1.0), forcing=0, film_is_B=True):
    """Periodic in x: A everywhere except a film of B (or the reverse) of `film` columns."""
    x = np.arange(nx)
    inside = (x >= (nx - film) // 2) & (x < (nx - film) // 2 + film)
    a_hi = ~inside if film_is_B else inside
    rA = np.repeat(np.where(a_hi, 1.0, 0.03)[None, :], ny, axis=0)
    rB = np.repeat(np.where(a_hi, 0.03, 1.0)[None, :], ny, axis=0)
    return dict(nx=nx, ny=ny, rhoA=rA, rhoB=rB, G_AB=3.0, G1=G1, G2=G2, tau=tau, forcing=forcing)


@pytest.mark.parametrize("case", ["droplet", "walls", "shift"])
def test_pressure_tensor_matches_oracle(torch, case):
    say("pressure parity", case)
    rng = np.random.default_rng(3)
    nx, ny = 70, 37
    yy, xx = np.mgrid[0:ny, 0:nx]
    disc = (xx - 33.2) ** 2 + (yy - 17.6) ** 2 <= 100
    d = dict(nx=nx, ny=ny, rhoA=np.where(disc, 1.0, 0.03) + 1e-3 * rng.standard_normal((ny, nx)),
             rhoB=np.where(disc, 0.03, 1.0), G_AB=3.0, G1=-7.4, G2=6.4, tau=(1.0, 0.8))
    if case == "walls":
        d.update(walls=1, rho_wall=(0.03, 1.0), g=((1e-5, 0.0), (1e-5, 0.0)))
    if case == "shift":
        d.update(forcing=1, tau=(1.0, 1.0))
    sim = lbm.Sim([d])
    sim.step(40)
    P, lt = sim.pressure()
    torch.cuda.synchronize()
    p = O.Params(nx=nx, ny=ny, G_AB=3.0, G1=-7.4, G2=6.4, tau=d["tau"], g=d.get("g", ((0, 0), (0, 0))),
                 walls=d.get("walls", 0), rho_wall=d.get("rho_wall", (0.0, 0.0)),
                 forcing=d.get("forcing", 0))
    Po = O.pressure(p, sim.populations_full())
    sim.close()
    err = np.linalg.norm(P.cpu().numpy() - Po) / np.linalg.norm(Po)
    lto = O.line_tension(Po)
    say("P rel err", err, "line tension", lt, lto)
    assert err < 1e-6
    assert abs(lt - lto) <= 1e-5 * np.abs(Po[0] - Po[1]).sum() / ny


def test_flat_interface_gamma_on_gpu(torch):
    """gamma of flat interfaces at the emulsion couplings (0.04, Sec. III D) and its
    independence of the viscosity ratio (within 1.2 % over M = 1/10, 1, 10, Sec. III C)."""
    say("flat gamma")
    # the oracle pin's slab (96 x 4, an A slab of 48 columns, 40000 steps): the bulk
    # densities of wider periodic slabs relax by diffusion only and take far longer
    gam = {}
    for M in (0.1, 1.0, 10.0):
        sim = lbm.Sim([slab_instance(96, 4, 48, -7.4, 6.4, tau=(1.0, 0.5 + 0.5 * M), film_is_B=False)])
        sim.step(40000)
        _, lt = sim.pressure()
        sim.close()
        gam[M] = lt / 2
        say("M", M, "gamma", gam[M])
    g1 = gam[1.0]
    assert abs(g1 - 0.04) / 0.04 < 0.10
    assert max(abs(v - g1) / g1 for v in gam.values()) <= 0.012, gam


def _film_instance(nx, ny, film, G1, G2, hi, lo):
    x = np.arange(nx)
    inside = (x >= (nx - film) // 2) & (x < (nx - film) // 2 + film)
    rA = np.repeat(np.where(inside, lo, hi)[None, :], ny, axis=0)
    rB = np.repeat(np.where(inside, hi, lo)[None, :], ny, axis=0)
    return dict(nx=nx, ny=ny, rhoA=rA, rhoB=rB, G_AB=3.0, G1=G1, G2=G2, tau=(1.0, 1.0))


def test_disjoining_pressure_shapes_of_fig3a(torch):
    """Eqs. 16-18 on films of B of thickness h between A (G_AB = 3.0), started at the
    coexistence densities of a long wide-slab run: the single-range case
    (G_A1 = G_A2 = 0) has a negative disjoining pressure at small h, the two-range
    cases a positive peak, higher for lower G_A1 (Fig. 3a and its caption)."""
    say("disjoining pressure")
    hs = [2, 3, 4, 5, 6, 8, 12, 24, 48]
    peak = {}
    for G1, G2 in ((0.0, 0.0), (-6.0, 5.0), (-8.0, 7.0)):
        sim = lbm.Sim([_film_instance(192, 4, 96, G1, G2, 1.0, 0.03)])
        sim.step(200000)
        r = sim.fields()[0].cpu().numpy()
        sim.close()
        hi, lo = float(r[0, 0, 0]), float(r[0, 0, 96])
        gf = []
        for h in hs + [128]:
            sim = lbm.Sim([_film_instance(h + 128, 4, h, G1, G2, hi, lo)])
            sim.step(60000)
            _, lt = sim.pressure()
            sim.close()
            gf.append(lt)
        gamma = gf.pop() / 2
        pis = O.disjoining_pressure(np.array(hs, float), np.array(gf), gamma) * 10.0 / gamma
        say("G", (G1, G2), "gamma", gamma, "Pi*", np.round(pis, 3).tolist())
        small = pis[:5]  # h <= 6
        peak[(G1, G2)] = small.max()
        if G1 == 0.0:
            assert small.min() < -0.3 and small.max() < 0.01, pis
    assert peak[(-6.0, 5.0)] > 0.05 and peak[(-8.0, 7.0)] > peak[(-6.0, 5.0)], peak


COLL_GAMMA = 0.043  # flat-interface gamma of the Sec. III D couplings (flat-gamma test above)


def collide(torch, G1, G2, tau, forcing=0, U=0.12, nx=320, ny=160, R=21, relax=3000,
            samples=16, every=500):
    """Two droplets of radius R relaxed at rest 10 nodes apart, then given velocities
    +-U/2 along x (equilibrium populations at the relaxed densities, the velocity
    weighted by the local A fraction so the matrix starts at rest).  Returns the
    droplet density and, per sample, (A regions with rho_A > 1/2, distance of the
    two halves' A centroids, largest rho_B in the gap on the axis)."""
    from scipy import ndimage
    yy, xx = np.mgrid[0:ny, 0:nx]
    cy, c1, c2 = ny // 2, nx / 2 - R - 5, nx / 2 + R + 5
    A = ((xx - c1) ** 2 + (yy - cy) ** 2 <= R * R) | ((xx - c2) ** 2 + (yy - cy) ** 2 <= R * R)
    sim = lbm.Sim([dict(nx=nx, ny=ny, rhoA=np.where(A, 1.0, 0.03), rhoB=np.where(A, 0.03, 1.0),
                        G_AB=3.0, G1=G1, G2=G2, tau=tau, forcing=forcing)])
    try:
        sim.step(relax)
        rho = sim.fields()[0].cpu().numpy().astype(np.float64)
        assert np.isfinite(rho).all()
        rho_drop = float(rho[0, cy, int(c1)])
        ux = np.where(xx < nx / 2, U / 2, -U / 2) * rho[0] / (rho[0] + rho[1])
        f = np.empty((2, 9, ny, nx))
        for k in range(2):
            for y in range(ny):
                for x in range(nx):
                    f[k, :, y, x] = O.feq(rho[k, y, x], ux[y, x], 0.0)
        w = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1]) / 36.0
        ref = np.asarray(sim.params[0].rho_ref[:])
        dev = f - w[None, :, None, None] * ref[:, None, None, None]
        sim.set_populations(torch.from_numpy(dev.astype(np.float32)).cuda())
        hist = []
        left = xx < nx / 2
        for _ in range(samples):
            sim.step(every)
            rho = sim.fields()[0].cpu().numpy().astype(np.float64)
            assert np.isfinite(rho).all()
            _, n = ndimage.label(rho[0] > 0.5)
            wA = rho[0] * (rho[0] > 0.5)
            xl = (wA * xx)[left].sum() / wA[left].sum()
            xr = (wA * xx)[~left].sum() / wA[~left].sum()
            gap = rho[1, cy - 2:cy + 3, nx // 2 - 3:nx // 2 + 4].max()
            hist.append((n, xr - xl, gap))
    finally:
        sim.close()
    return rho_drop, hist


@pytest.mark.parametrize("M", [1, 3])
def test_droplet_collision_bounces_at_both_viscosity_ratios(torch, M):
    """Present model, mu_A = 0.1 (tau_A = 0.8), mu_B = M mu_A (Figs. 5b, 6b)."""
    say("collision present M", M)
    tau = (0.8, 0.5 + 0.3 * M)
    R, U = 21, 0.12
    rho_drop, hist = collide(torch, -7.4, 6.4, tau, U=U, R=R)
    say("rho_A", rho_drop, "samples", [(n, round(s, 1), round(g, 3)) for n, s, g in hist])
    mu_A = rho_drop * (tau[0] - 0.5) / 3.0
    Ca, We = mu_A * U / COLL_GAMMA, rho_drop * 2 * R * U * U / COLL_GAMMA
    assert 0.25 < Ca < 0.35 and 12.0 < We < 18.0, (Ca, We)
    sep = [s for _, s, _ in hist]
    assert all(n == 2 for n, _, _ in hist), hist
    assert all(g > 0.5 for _, _, g in hist), hist  # the film of B is never drained
    smin = min(sep)
    assert smin < 2 * R, sep  # the droplets met and flattened against the film
    assert sep[-1] > smin + 10.0 and sep.index(smin) < len(sep) // 2, sep  # and bounced back


def test_droplet_collision_coalesces_without_the_two_range_interaction(torch):
    """Single-range model (G_A1 = G_A2 = 0), same collision: the film drains."""
    say("collision single-range")
    _, hist = collide(torch, 0.0, 0.0, (0.8, 0.8))
    say("samples", [(n, round(s, 1), round(g, 3)) for n, s, g in hist])
    n, _, gap = hist[-1]
    assert n == 1 and gap < 0.3, hist


def test_droplet_collision_original_model_bounces_at_unit_ratio(torch):
    """Original model (velocity shift), M = 1 (Fig. 5a).  At mu_A = 0.1 these couplings
    diverge under the velocity shift (the FP64 oracle as well), so tau = 1 here."""
    say("collision original M 1")
    _, hist = collide(torch, -7.4, 6.4, (1.0, 1.0), forcing=1)
    say("samples", [(n, round(s, 1), round(g, 3)) for n, s, g in hist])
    sep = [s for _, s, _ in hist]
    assert all(n == 2 for n, _, _ in hist) and all(g > 0.5 for _, _, g in hist), hist
    assert sep[-1] > min(sep) + 10.0, sep


def emulsion_cases(L, R_list, tau=1.0, Fbar=37.0):
    """Walled L x L channels, one per R (R = 0: no droplets), each holding 5 x 5
    droplets of A of radius R on a square grid in the B matrix; the body force
    F_b = Fbar 8 nu^2 / L^3 on both components (Fbar = F_b L^3 / (8 rho nu^2) as
    in Sec. III D, rho_B = 1)."""
    nu = (tau - 0.5) / 3.0
    Fb = Fbar * 8.0 * nu * nu / L ** 3
    yy, xx = np.mgrid[0:L, 0:L]
    out = []
    for R in R_list:
        A = np.zeros((L, L), bool)
        for i in range(5 if R else 0):
            for j in range(5):
                A |= (xx - (i + 0.5) * L / 5) ** 2 + (yy - (j + 0.5) * L / 5) ** 2 <= R * R
        out.append((float(A.mean()), dict(nx=L, ny=L, rhoA=np.where(A, 1.0, 0.03),
                                          rhoB=np.where(A, 0.03, 1.0), G_AB=3.0, G1=-7.4, G2=6.4,
                                          tau=(tau, tau), walls=1, rho_wall=(0.03, 1.0),
                                          g=((0.0, 0.0), (0.0, 0.0)))))
    return Fb, nu, out


def test_emulsion_relative_viscosity_follows_the_fit(torch):
    """The droplets relax 30 000 steps at rest, then the body force drives the
    channel for 270 000 steps (about nine decay times L^2 / (pi^2 nu) of the
    slowest viscous mode)."""
    import time
    L = 220
    Fb, nu, cases = emulsion_cases(L, (0.0, 10.0, 12.5, 15.0))
    say("emulsion", L, "phi", [round(p, 3) for p, _ in cases])
    sim = lbm.Sim([c for _, c in cases])
    try:
        t0 = time.time()
        sim.step(30000)
        for i in range(len(cases)):
            p = lbm.lbm_params.from_buffer_copy(sim.params[i])
            p.g[0][0] = Fb
            p.g[1][0] = Fb
            lbm.lbm_set_params(sim.ctx, i, p)
            sim.params[i] = p
        sim.step(270000)
        obs, _ = sim.observables()
        rho = [sim.fields(i)[0].cpu().numpy() for i in range(len(cases))]
        say("emulsion steps done in", round(time.time() - t0, 1), "s")
    finally:
        sim.close()
    assert all(o["finite"] for o in obs)
    Q = [o["flow_rate"] for o in obs]
    phi = [p for p, _ in cases]
    mu = [Q[0] / q for q in Q]
    demt = [(1.0 - p) ** -0.88 for p in phi]
    say("Q", [round(q, 4) for q in Q], "mu_r", [round(m, 4) for m in mu],
        "DEMT", [round(d, 4) for d in demt])
    # no droplets: plane Poiseuille flow between half-way walls, Q = F_b L^3 / (12 nu)
    # per unit density (Sec. III D defines Fbar with the matrix density)
    q_pois = Fb * L ** 3 / (12.0 * nu)
    assert abs(Q[0] / q_pois - 1.0) < 0.01, (Q[0], q_pois)
    assert all(b > a for a, b in zip(mu, mu[1:])), mu
    for m, d in zip(mu[1:], demt[1:]):
        assert abs(m / d - 1.0) < 0.10, (mu, demt)
    for (p, _), r in zip(cases[1:], rho[1:]):  # the droplets neither dissolve nor grow
        assert abs(float((r[0] > 0.5).mean()) / p - 1.0) < 0.1, (p, float((r[0] > 0.5).mean()))
