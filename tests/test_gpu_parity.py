"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Tolerances are norm-wise relative errors ||gpu - oracle||_2 / ||oracle||_2 of
the density and barycentric-velocity fields, as the precision form of the
method states them (<= 1e-5 after 1000 steps of the 64x64 droplet with its
literal couplings); other cases carry the bound derived for them in the
design notes.  Integer-like results (batched vs single runs, graph vs
launch-by-launch, repeated runs) must be bitwise equal.
"""
import dataclasses
import math
import random
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as O
from paper_1806_06943_amd import lbm, tune
from paper_1806_06943_amd import workloads as W
from tests.exact_forces import forces_exact

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


def oparams(w):
    return O.Params(nx=w.nx, ny=w.ny, G_AB=w.G_AB, G1=w.G1, G2=w.G2, tau=w.tau, g=w.g,
                    walls=w.walls, rho_wall=w.rho_wall)


def run_pair(torch, w, steps):
    """GPU and oracle after `steps` steps from the same initial densities."""
    say("run_pair", w.name, w.nx, w.ny, "steps", steps)
    sim = lbm.Sim([lbm.workload_instance(w)])
    sim.step(steps)
    rho, u = sim.fields()
    p = oparams(w)
    fo = O.run(p, O.init(p, w.rhoA, w.rhoB), steps)
    return sim, rho.cpu().numpy(), u.cpu().numpy(), p, fo


# ---------------------------------------------------------------- forces alone
@pytest.mark.parametrize("nx,ny,walls,seed", [(4, 4, False, 11), (5, 3, False, 12),
                                              (4, 6, True, 13), (70, 9, False, 14)])
def test_forces_exact_bruteforce(torch, nx, ny, walls, seed):
    """The step's force code against exact-rational sums of Eqs. 8, 9 (tiles wider
    than the lattice alias the +-2 offsets)."""
    say("forces bruteforce", nx, ny, walls)
    r = random.Random(seed)
    rho = [[[Fr(r.randint(20, 1200), 1024) for _ in range(nx)] for _ in range(ny)] for _ in range(2)]
    rho32 = np.array([[[float(v) for v in row] for row in rho[k]] for k in range(2)], dtype=np.float32)
    # psi exactly as the kernel computes it is unknown to rounding; use FP64 psi of the FP32 rho
    psi = [[[Fr(-math.expm1(-float(v))) for v in row] for row in rho[k]] for k in range(2)]
    rho_wall = (0.03, 1.0)
    g = ((Fr(1, 4096), Fr(-1, 8192)), (Fr(3, 8192), Fr(1, 2048)))
    Fx = forces_exact(nx, ny, rho, psi, Fr(-7.4), Fr(6.4), Fr(3.0), g=g, walls=walls,
                      rho_wall=tuple(Fr(v) for v in rho_wall),
                      psi_wall=tuple(Fr(-math.expm1(-v)) for v in rho_wall))
    exact = np.array([[[[float(v) for v in row] for row in Fx[k][d]] for d in range(2)] for k in range(2)])
    sim = lbm.Sim([dict(nx=nx, ny=ny, rhoA=rho32[0], rhoB=rho32[1], G_AB=3.0, G1=-7.4, G2=6.4,
                        tau=(1.0, 0.6), walls=int(walls), rho_wall=rho_wall,
                        g=tuple(tuple(float(v) for v in gk) for gk in g))])
    F = sim.forces(torch.from_numpy(rho32).cuda()).cpu().numpy()
    scale = np.abs(exact).max()
    # FP32: psi rounding (1 ulp of ~0.7) times the merged weights, |sum c e| ~ 1.2, times psi
    assert np.abs(F - exact).max() <= 2e-6 * max(scale, 1.0)


def test_forces_sinusoid_closed_form(torch):
    """psi = a + b sin(kx): sum_i w_i psi(x+e_i) e_ix = (b/3) sin k cos kx (Eq. 8 first belt)."""
    nx, ny, m = 96, 5, 3
    k = 2 * math.pi * m / nx
    x = np.arange(nx)
    a, b = 0.4, 0.1
    psi = np.tile(a + b * np.sin(k * x), (ny, 1))
    rho = (-np.log1p(-psi)).astype(np.float32)
    sim = lbm.Sim([dict(nx=nx, ny=ny, rhoA=rho, rhoB=rho, G_AB=0.0, G1=1.0, G2=0.0, tau=(1.0, 1.0))])
    F = sim.forces(torch.from_numpy(np.stack([rho, rho])).cuda()).cpu().numpy()
    expect = -psi[0] * (b / 3) * math.sin(k) * np.cos(k * x)
    assert np.abs(F[0, 0] - expect).max() < 1e-7
    assert np.abs(F[0, 1]).max() < 1e-7


# ---------------------------------------------------------------- one step
@pytest.mark.parametrize("walls", [0, 1])
def test_single_step_matches_oracle(torch, walls):
    """One GPU step from a developed state equals one oracle step of the same (FP32) state."""
    say("single step walls", walls)
    if walls:
        w = W.emulsion(nx=80, ny=40, ndrop=2, radius=8, gx=1e-5)
    else:
        w = W.droplet(nx=80, ny=72, radius=14, couplings=W.COUPLINGS_PAPER)
    p = oparams(w)
    f = O.run(p, O.init(p, w.rhoA, w.rhoB), 60)
    sim = lbm.Sim([lbm.workload_instance(w)])
    ref = np.asarray(sim.params[0].rho_ref[:])
    wts = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1]) / 36.0
    dev = (f - wts[None, :, None, None] * ref[:, None, None, None]).astype(np.float32)
    sim.set_populations(torch.from_numpy(dev).cuda())
    f32 = dev.astype(np.float64) + wts[None, :, None, None] * ref[:, None, None, None]
    sim.step(1)
    got = sim.populations_full()
    want = O.step(p, f32)
    err = np.abs(got - want).max()
    assert err < 2e-7, err


# ---------------------------------------------------------------- 1000 steps of the droplet
def test_droplet_1000_steps_literal_couplings(torch):
    """64x64 droplet, G_AB=0.405, G1=-9.0, G2=8.1, tau=(1.0, 0.6): <= 1e-5 on rho_A, rho_B, u."""
    w = W.droplet()
    sim, rho, u, p, fo = run_pair(torch, w, 1000)
    flo = O.fields(p, fo)
    errs = [rel(rho[0], flo["rho"][0]), rel(rho[1], flo["rho"][1]),
            rel(u[0], flo["u"][0]), rel(u[1], flo["u"][1])]
    say("literal errors", errs)
    assert max(errs) <= 1e-5, errs
    # the GPU state itself, evaluated by the oracle
    fl_state = O.fields(p, sim.populations_full())
    assert rel(fl_state["u"], flo["u"]) <= 1e-5


def test_droplet_1000_steps_paper_couplings(torch):
    """Same droplet with the demixing couplings of the emulsion section (3.0, -7.4, 6.4):
    sharp interfaces amplify FP32 rounding; bound 5e-5 on u, 1e-5 on densities."""
    w = W.droplet(couplings=W.COUPLINGS_PAPER)
    sim, rho, u, p, fo = run_pair(torch, w, 1000)
    flo = O.fields(p, fo)
    er = [rel(rho[0], flo["rho"][0]), rel(rho[1], flo["rho"][1])]
    eu = [rel(u[0], flo["u"][0]), rel(u[1], flo["u"][1])]
    say("paper errors", er, eu)
    assert max(er) <= 1e-5 and max(eu) <= 5e-5, (er, eu)


def test_walled_emulsion_crop(torch):
    """Walled channel with body force (a 128x64 crop of the emulsion workload), 2000 steps."""
    w = W.emulsion(nx=128, ny=64, ndrop=3, radius=10, gx=1e-5)
    sim, rho, u, p, fo = run_pair(torch, w, 2000)
    flo = O.fields(p, fo)
    er = [rel(rho[0], flo["rho"][0]), rel(rho[1], flo["rho"][1])]
    eu = [rel(u[0], flo["u"][0]), rel(u[1], flo["u"][1])]
    say("walls errors", er, eu)
    assert max(er) <= 1e-5 and max(eu) <= 5e-5, (er, eu)


# ---------------------------------------------------------------- observables
def test_observables_match_oracle(torch):
    """FP64 reductions on the device against the oracle's observables of its own state."""
    w = W.droplet(couplings=W.COUPLINGS_PAPER)
    sim, rho, u, p, fo = run_pair(torch, w, 1000)
    obs, ubar = sim.observables()
    o = obs[0]
    flo = O.fields(p, fo)
    L = O.laplace(p, flo)
    m0 = O.masses(O.init(p, w.rhoA, w.rhoB))
    assert np.allclose(o["mass"], m0, rtol=1e-6, atol=0)
    assert abs(o["R_eff"] - L["R"]) / L["R"] < 1e-5
    assert abs(o["cx"] - L["cx"]) < 1e-3 and abs(o["cy"] - L["cy"]) < 1e-3
    assert abs(o["n_in"] - L["n_in"]) <= 2 and abs(o["n_out"] - L["n_out"]) <= 4
    assert abs(o["dp"] - L["dp"]) / abs(L["dp"]) < 1e-3
    assert abs(o["max_speed"] - O.max_speed(flo)) / O.max_speed(flo) < 1e-4
    row = flo["rho"][0][int(math.floor(L["cy"] + 0.5)) % p.ny]
    Wo = O.interface_width_row(row, int(math.floor(L["cx"] + 0.5)) % p.nx)
    assert abs(o["width"] - Wo) / Wo < 1e-4
    assert np.allclose(ubar, O.flow_profile(flo), rtol=0, atol=1e-7)
    assert o["finite"] == 1


def test_nonfinite_state_is_reported(torch):
    w = W.droplet(nx=32, ny=32, radius=6)
    w.rhoA[5, 7] = float("nan")
    sim = lbm.Sim([lbm.workload_instance(w, rho_ref=(0.1, 0.9))])
    sim.step(3)
    obs, _ = sim.observables(check=False)
    assert sim.last_rc == lbm.LBM_ENONFINITE and obs[0]["finite"] == 0


# ---------------------------------------------------------------- determinism, graphs, batching
def test_graph_replay_equals_launches_and_is_deterministic(torch):
    """Every replay of the captured 16-step graph, with eager work (observables,
    fields, a population export) and synchronisations between the replays, equals
    16 single launches bitwise."""
    w = W.droplet(couplings=W.COUPLINGS_PAPER)
    a = lbm.Sim([lbm.workload_instance(w)])
    b = lbm.Sim([lbm.workload_instance(w)])
    for replay in range(3):
        a.step(16)              # one graph replay
        for _ in range(16):     # launch by launch
            b.step(1)
        fa, fb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
        assert np.array_equal(fa, fb), replay
        a.observables()
        a.fields()
        torch.cuda.synchronize()
    c = lbm.Sim([lbm.workload_instance(w)])
    c.step(37)
    c.step(11)
    assert np.array_equal(c.populations().cpu().numpy(), fa)


def test_zero_step_calls_change_nothing(torch):
    """Empty work: zero steps, a recording of zero steps (no store needed) and an
    adjoint run of zero steps leave the state, the step count and lambda as they were."""
    w = W.droplet(nx=40, ny=24, radius=6, couplings=W.COUPLINGS_PAPER)
    sim = lbm.Sim([lbm.workload_instance(w)])
    try:
        sim.step(5)
        f0, n0 = sim.populations().clone(), sim.steps_done
        sim.step(0)
        lbm.lbm_record(sim.ctx, 0, 0, 0)
        lam = torch.randn((2, 9, 24, 40), dtype=torch.float32, device=f0.device)
        lam0, tmp = lam.clone(), torch.empty_like(lam)
        grad = torch.zeros(5, dtype=torch.float64, device=f0.device)
        lbm.lbm_adjoint_run(sim.ctx, 0, 0, 0, lam.data_ptr(), tmp.data_ptr(), grad.data_ptr())
        torch.cuda.synchronize()
        assert torch.equal(sim.populations(), f0) and sim.steps_done == n0
        assert torch.equal(lam, lam0) and not grad.any()
    finally:
        sim.close()


def test_batched_instances_equal_single_runs(torch):
    """One launch over uneven instances gives each instance's single-run result bitwise."""
    ws = [W.droplet(nx=64, ny=64, radius=10, couplings=W.COUPLINGS_PAPER),
          W.emulsion(nx=96, ny=40, ndrop=2, radius=8, gx=1e-5),
          W.droplet(nx=40, ny=72, radius=9, couplings=W.COUPLINGS_LITERAL, tau=(1.6, 1.0), sub=3)]
    batch = lbm.Sim([lbm.workload_instance(w) for w in ws])
    batch.step(100)
    for i, w in enumerate(ws):
        single = lbm.Sim([lbm.workload_instance(w)])
        single.step(100)
        assert np.array_equal(batch.populations(i).cpu().numpy(), single.populations().cpu().numpy()), i


# ---------------------------------------------------------------- full size, sampled
def test_spinodal_full_size_sampled_nodes(torch):
    """2048x2048 spinodal workload in the benchmark's launch configuration (the tuned
    strip plan): sampled nodes of step t+1 against the oracle's single-node step of the
    GPU state at t; FP64 mass."""
    w = W.spinodal()
    say("spinodal 2048^2")
    sim = lbm.Sim([lbm.workload_instance(w)])
    tune.tune(sim, use_cache=False, nrep=5)
    say("plan", lbm.lbm_get_strip_width(sim.ctx),
        lbm.lbm_get_tiling(sim.ctx), lbm.lbm_get_balance(sim.ctx))
    obs0, _ = sim.observables()
    sim.step(64)
    f = sim.populations_full()
    sim.step(1)
    f1 = sim.populations_full()
    p = oparams(w)
    r = np.random.default_rng(7)
    nodes = [(0, 0), (2047, 2047), (0, 2047), (2047, 0), (1024, 3)] + \
            [tuple(int(v) for v in r.integers(0, 2048, size=2)) for _ in range(40)]
    for x, y in nodes:
        want = O.step_at(p, f, x, y)
        assert np.abs(f1[:, :, y, x] - want).max() < 2e-7, (x, y)
    sim.step(200)
    obs1, _ = sim.observables()
    for k in range(2):
        assert abs(obs1[0]["mass"][k] - obs0[0]["mass"][k]) / obs0[0]["mass"][k] < 1e-6


def test_largest_lattice_sampled_nodes(torch):
    """The largest lattice the library accepts at nx = 64 (466033 rows: population
    byte offsets up to 2 GiB less 3 KiB inside one buffer), walled, with a layer and
    droplets of A, under a one-wavefront and a two-wavefront strip plan: sampled nodes
    of step t+1, the last rows included, against the oracle's single-node step of the
    GPU state at t; FP64 mass."""
    nx, ny = 64, 466033
    say("largest lattice", nx, ny)
    rng = np.random.default_rng(5)
    yy, xx = np.arange(ny)[:, None], np.arange(nx)[None, :]
    A = (((yy >= ny - 40) & (yy < ny - 20)) | ((xx - 32) ** 2 + (yy - 20) ** 2 <= 100) |
         ((xx - 20) ** 2 + (yy - ny // 2) ** 2 <= 144))
    A = np.broadcast_to(A, (ny, nx))
    cp = dict(G_AB=3.0, G1=-7.4, G2=6.4, tau=(1.0, 0.7), walls=1, rho_wall=(0.03, 1.0),
              g=((1e-5, 0.0), (1e-5, 0.0)))
    inst = dict(nx=nx, ny=ny, rhoA=np.where(A, 1.0, 0.03) + rng.uniform(-1e-3, 1e-3, (ny, nx)),
                rhoB=np.where(A, 0.03, 1.0) + rng.uniform(-1e-3, 1e-3, (ny, nx)), **cp)
    p = O.Params(nx=nx, ny=ny, **cp)
    nodes = [(0, ny - 1), (63, ny - 1), (31, ny - 2), (5, ny - 3), (17, ny - 30), (0, 0), (63, 0),
             (32, 20), (20, ny // 2), (44, ny // 2 + 11)] + \
            [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(10)]
    for cols, h in ((58, 74), (122, 512)):
        sim = lbm.Sim([inst])
        try:
            lbm.lbm_set_strip_width(sim.ctx, cols)
            lbm.lbm_set_tiling(sim.ctx, h)
            obs0, _ = sim.observables()
            sim.step(3)
            f = sim.populations_full()
            sim.step(1)
            f1 = sim.populations_full()
            for x, y in nodes:
                want = O.step_at(p, f, x, y)
                assert np.abs(f1[:, :, y, x] - want).max() < 2e-7, (cols, x, y)
            del f, f1
            sim.step(4)
            obs1, _ = sim.observables()
            for k in range(2):
                assert abs(obs1[0]["mass"][k] - obs0[0]["mass"][k]) / obs0[0]["mass"][k] < 1e-6
        finally:
            sim.close()


@pytest.mark.parametrize("ratio", [0.5, 1.0, 2.0, 4.0])
def test_emulsion_full_size_sampled_nodes(torch, ratio):
    """4096x512 walled emulsion (200 droplets, g_x = 1e-6, nu_A/nu_B = ratio) under the
    tuned strip plan: sampled nodes, wall rows and lattice edges included, of step t+1
    against the oracle's single-node step; FP64 mass of each component."""
    w = W.emulsion(tau_ratio=ratio)
    say("emulsion 4096x512 ratio", ratio)
    sim = lbm.Sim([lbm.workload_instance(w)])
    tune.tune(sim, use_cache=False, nrep=5)
    obs0, _ = sim.observables()
    sim.step(48)
    f = sim.populations_full()
    sim.step(1)
    f1 = sim.populations_full()
    p = oparams(w)
    r = np.random.default_rng(11)
    nodes = [(0, 0), (4095, 511), (0, 511), (4095, 0), (2048, 1), (17, 510)] + \
            [(int(r.integers(0, 4096)), int(y)) for y in r.integers(0, 512, size=30)] + \
            [(int(r.integers(0, 4096)), y) for y in (0, 1, 510, 511) for _ in range(3)]
    for x, y in nodes:
        want = O.step_at(p, f, x, y)
        assert np.abs(f1[:, :, y, x] - want).max() < 2e-7, (x, y)
    sim.step(151)
    obs1, _ = sim.observables()
    for k in range(2):
        assert abs(obs1[0]["mass"][k] - obs0[0]["mass"][k]) / obs0[0]["mass"][k] < 1e-6


def test_batched_workload_per_instance_laplace(torch):
    """The 96-instance droplet batch in one context under its tuned plan, 300 steps: one
    instance of each size against a full oracle run (fields, and the Laplace pressure
    jump of Sec. III B by the same protocol)."""
    ws = W.batched()
    say("batched 96 instances")
    sim = lbm.Sim([lbm.workload_instance(w) for w in ws])
    tune.tune(sim, use_cache=False, nrep=5)
    steps = 300
    sim.step(steps)
    obs, _ = sim.observables()
    seen = set()
    for i, w in enumerate(ws):
        if w.nx in seen:
            continue
        seen.add(w.nx)
        say("instance", i, w.nx, w.tau, w.G2)
        rho, u = sim.fields(i)
        p = oparams(w)
        fo = O.run(p, O.init(p, w.rhoA, w.rhoB), steps)
        flo = O.fields(p, fo)
        er = [rel(rho.cpu().numpy()[k], flo["rho"][k]) for k in range(2)]
        eu = [rel(u.cpu().numpy()[d], flo["u"][d]) for d in range(2)]
        assert max(er) <= 1e-5 and max(eu) <= 5e-5, (i, er, eu)
        L = O.laplace(p, flo)
        assert abs(obs[i]["dp"] - L["dp"]) <= 1e-3 * abs(L["dp"]), (i, obs[i]["dp"], L["dp"])
        assert abs(obs[i]["R_eff"] - L["R"]) <= 1e-4 * L["R"]
    assert len(seen) == 4


# ---------------------------------------------------------------- geometry edge cases
@pytest.mark.parametrize("nx,ny,walls", [(4, 4, 0), (5, 3, 0), (1, 8, 0), (3, 7, 1), (70, 3, 0),
                                         (63, 5, 1), (125, 9, 0), (2, 1, 0)])
def test_small_and_ragged_lattices(torch, nx, ny, walls):
    """Lattices narrower than a strip (offsets alias), one-column and one-row tori,
    walls on a few rows, ragged strip widths: 40 steps against the oracle."""
    say("small lattice", nx, ny, walls)
    r = np.random.default_rng(nx * 100 + ny)
    rhoA = 0.5 + r.uniform(-0.2, 0.2, size=(ny, nx))
    rhoB = 0.5 + r.uniform(-0.2, 0.2, size=(ny, nx))
    inst = dict(nx=nx, ny=ny, rhoA=rhoA, rhoB=rhoB, G_AB=3.0, G1=-7.4, G2=6.4, tau=(1.0, 0.7),
                walls=walls, rho_wall=(0.3, 0.6), g=((1e-4, 2e-5), (1e-4, 2e-5)))
    sim = lbm.Sim([inst])
    sim.step(40)
    p = O.Params(nx=nx, ny=ny, G_AB=3.0, G1=-7.4, G2=6.4, tau=(1.0, 0.7), walls=walls,
                 rho_wall=(0.3, 0.6), g=((1e-4, 2e-5), (1e-4, 2e-5)))
    fo = O.run(p, O.init(p, rhoA, rhoB), 40)
    got = sim.populations_full()
    assert rel(got, fo) < 1e-6
    assert np.abs(got - fo).max() < 1e-6


@pytest.mark.parametrize("width", [506, 240, 122, 58])
def test_fitted_heights_sit_just_under_cu_multiples(torch, width):
    """The tuner's fitted heights: at h the launch has at most k CUs' worth of
    workgroups, at h - 1 more (2048 x 2048 lattice; host planning only)."""
    w = W.spinodal(nx=2048, ny=2048)
    sim = lbm.Sim([lbm.workload_instance(w)])
    ncu = tune._ncu(sim)
    hs = tune.fitted_heights(sim, width, ncu)
    assert hs
    for h in hs:
        tune.apply(sim, width, h)
        n = lbm.lbm_get_workgroups(sim.ctx)
        k = -(-n // ncu)
        assert n <= k * ncu
        if h > tune.MIN_HEIGHT:
            tune.apply(sim, width, h - 1)
            assert lbm.lbm_get_workgroups(sim.ctx) > k * ncu, (h, n)
    sim.close()


def test_strip_height_does_not_change_results(torch):
    """The strip height only moves work between wavefronts: results are bitwise equal."""
    w = W.emulsion(nx=200, ny=96, ndrop=4, radius=9, gx=1e-5)
    ref = None
    for h in (2, 3, 4, 7, 16, 40, 96):
        sim = lbm.Sim([lbm.workload_instance(w)])
        lbm.lbm_set_tiling(sim.ctx, h)
        assert lbm.lbm_get_tiling(sim.ctx) == h
        sim.step(35)
        f = sim.populations().cpu().numpy()
        if ref is None:
            ref = f
        assert np.array_equal(f, ref), h


def test_strip_heights_past_15_bits(torch):
    """A segment height is packed beside its width as an unsigned 16-bit field:
    chunks of 32768 rows and more (the word's sign bit set) advance the same
    rows as short chunks, bit for bit, on a tall, narrow walled lattice."""
    ny = 40000
    say("tall chunks", 16, ny)
    rA = np.full((ny, 16), 0.03)
    rA[ny // 4: 3 * ny // 4, 4:12] = 1.0
    rA += 1e-3 * np.random.default_rng(3).random((ny, 16))
    inst = dict(nx=16, ny=ny, rhoA=rA, rhoB=1.03 - rA, G_AB=3.0, G1=-7.4, G2=6.4,
                tau=(1.0, 0.6), walls=1, rho_wall=(0.03, 1.0), g=((1e-5, 0.0), (1e-5, 0.0)))
    ref = None
    for h in (16, 32768, 40000, 65535):
        sim = lbm.Sim([inst])
        lbm.lbm_set_tiling(sim.ctx, h)
        assert lbm.lbm_get_workgroups(sim.ctx) == -(-ny // h), h
        sim.step(5)
        f = sim.populations().cpu().numpy()
        sim.close()
        if ref is None:
            ref = f
        assert np.array_equal(f, ref), h


FULL_ROW_CASES = {
    "64x40": [(64, 40, 0)],
    "128x33w": [(128, 33, 1)],
    "192x50": [(192, 50, 0)],
    "256x24w": [(256, 24, 1)],
    "320x17": [(320, 17, 0)],
    "512x9w": [(512, 9, 1)],
    "64x1": [(64, 1, 0)],
    "mixed": [(64, 64, 0), (128, 40, 1), (192, 30, 0), (256, 20, 1), (64, 7, 1)],
}


def full_row_instances(spec, forcing=0):
    out = []
    for j, (nx, ny, walls) in enumerate(spec):
        r = np.random.default_rng(1000 + 17 * j + nx + ny)
        yy, xx = np.mgrid[0:ny, 0:nx]
        disc = (xx - nx / 3) ** 2 + (yy - ny / 2) ** 2 <= (min(nx, ny) / 3) ** 2
        rA = np.where(disc, 1.0, 0.03) + r.uniform(-1e-3, 1e-3, (ny, nx))
        rB = np.where(disc, 0.03, 1.0) + r.uniform(-1e-3, 1e-3, (ny, nx))
        out.append(dict(nx=nx, ny=ny, rhoA=rA, rhoB=rB, G_AB=3.0, G1=-7.4, G2=6.4,
                        tau=(1.0, 1.0) if forcing else (1.0, 0.7), walls=walls,
                        rho_wall=(0.03, 1.0), g=((2e-5, 1e-6), (2e-5, 1e-6)), forcing=forcing))
    return out


@pytest.mark.parametrize("case", sorted(FULL_ROW_CASES))
def test_full_row_plans_equal_strip_plans(torch, case):
    """Full-row plans (groups of nx / 64 wavefronts covering whole rows, several
    groups per workgroup) give the strip plans' results bit for bit: lattice
    widths 64 to 512, walls, one-row tori, mixed widths in one context, chunk
    heights from 2 rows to whole lattices; for the velocity shift too."""
    say("full rows", case)
    for forcing in (0, 1):
        insts = full_row_instances(FULL_ROW_CASES[case], forcing)
        ref = None
        for h in (0, 2, 3, 5, 16, 65535):
            sim = lbm.Sim(insts)
            if h:
                lbm.lbm_set_tiling(sim.ctx, h)
                lbm.lbm_set_full_rows(sim.ctx, 1)
                assert lbm.lbm_get_full_rows(sim.ctx) == 1
            sim.step(21)
            f = [sim.populations(i).cpu().numpy() for i in range(len(insts))]
            sim.close()
            if ref is None:
                ref = f
            for i in range(len(insts)):
                assert np.array_equal(f[i], ref[i]), (case, forcing, h, i)


def test_full_row_recording_equals_strip_recording(torch):
    """A recorded window (the step's override buffers, densities written) under a
    full-row plan stores the same states as under a strip plan, bit for bit."""
    insts = full_row_instances([(128, 48, 1), (64, 30, 0)])
    stores = []
    for fr in (0, 1):
        sim = lbm.Sim(insts)
        if fr:
            lbm.lbm_set_tiling(sim.ctx, 7)
            lbm.lbm_set_full_rows(sim.ctx, 1)
        sim.step(5)
        n = lbm.lbm_record_floats(sim.ctx, 0)
        S = torch.zeros((6, n), dtype=torch.float32, device="cuda:0")
        lbm.lbm_record(sim.ctx, 0, 5, S.data_ptr())
        torch.cuda.synchronize()
        stores.append((S.cpu().numpy(), sim.populations(0).cpu().numpy(), sim.populations(1).cpu().numpy()))
        sim.close()
    # a slot: populations (18 ny pitch floats, padded by 64) then densities
    # (2 ny pitch, padded by 64); the pads hold whatever the workspace held
    nf, nr = 18 * 48 * 128, 2 * 48 * 128
    for a, b in ((stores[0][0], stores[1][0]),):
        assert a.shape[1] == nf + 64 + nr + 64
        assert np.array_equal(a[:5, :nf], b[:5, :nf])
        assert np.array_equal(a[:5, nf + 64:nf + 64 + nr], b[:5, nf + 64:nf + 64 + nr])
    for j in (1, 2):
        assert np.array_equal(stores[0][j], stores[1][j])


def test_full_rows_refused_for_other_widths(torch):
    w = W.droplet(nx=96, ny=64)
    sim = lbm.Sim([lbm.workload_instance(w)])
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_set_full_rows(sim.ctx, 1)
    assert ei.value.code == lbm.LBM_EUNSUPPORTED
    assert lbm.lbm_get_full_rows(sim.ctx) == 0
    sim.close()


def test_batched_workload_full_rows_equal_strips(torch):
    """The 96-instance droplet batch under its strip plan and under full-row plans."""
    ws = W.batched()
    insts = [lbm.workload_instance(w) for w in ws]
    ref = None
    for fr, h in ((0, 64), (1, 64), (1, 21)):
        sim = lbm.Sim(insts)
        lbm.lbm_set_tiling(sim.ctx, h)
        if fr:
            lbm.lbm_set_full_rows(sim.ctx, 1)
        sim.step(40)
        f = [sim.populations(i).cpu().numpy() for i in (0, 1, 2, 5, 50, 95)]
        sim.close()
        if ref is None:
            ref = f
        for a, b in zip(f, ref):
            assert np.array_equal(a, b), (fr, h)


@pytest.mark.parametrize("nx,ny,walls", [(200, 96, 1), (600, 40, 0), (37, 21, 1)])
def test_strip_width_does_not_change_results(torch, nx, ny, walls):
    """Strips of 1 to 8 wavefronts, balanced or 64-byte aligned, uniform chunks or an
    equal share of rows per workgroup: bitwise equal results (wider lattices than one
    strip exercise the exchange between wavefronts)."""
    say("strip widths", nx, ny, walls)
    if walls and ny >= 60:
        w = W.emulsion(nx=nx, ny=ny, ndrop=3, radius=6, gx=1e-5)
    else:
        w = W.droplet(nx=nx, ny=ny, radius=min(nx, ny) / 4)
        if walls:
            w = dataclasses.replace(w, walls=1, rho_wall=(0.03, 1.0), g=((1e-5, 0.0), (1e-5, 0.0)))
    ref = None
    # (cols, rows or -balance): uniform plans, then balanced plans (1-4 workgroups per CU)
    for cols, h in ((58, 16), (48, 8), (122, 12), (112, 5), (250, 16), (240, 33), (506, 7), (496, 16),
                    (16, 4), (240, -2), (58, -1), (506, -3), (48, -4), (122, -2)):
        sim = lbm.Sim([lbm.workload_instance(w)])
        lbm.lbm_set_strip_width(sim.ctx, cols)
        if h > 0:
            lbm.lbm_set_tiling(sim.ctx, h)
        else:
            lbm.lbm_set_balance(sim.ctx, -h)
            assert lbm.lbm_get_balance(sim.ctx) == -h
        assert lbm.lbm_get_strip_width(sim.ctx) == cols
        sim.step(23)
        f = sim.populations().cpu().numpy()
        sim.close()
        if ref is None:
            ref = f
        assert np.array_equal(f, ref), (cols, h)


def test_density_calls_follow_the_state(torch):
    """The step moves only populations; the calls that read densities compute those
    of the current state (a recording writes them itself).  A context taken
    through steps, a force evaluation (which uses a scratch density buffer), a
    recorded window and changes of strip plan (uniform, balanced) stays bitwise
    equal to one stepped plainly, and its fields equal those of a context into
    which the same populations were imported.  Strips wider than a workgroup of
    eight wavefronts covers (506 output columns) are refused."""
    say("density calls")
    w = dataclasses.replace(W.droplet(nx=96, ny=40, radius=10), walls=1, rho_wall=(0.03, 1.0),
                            g=((1e-5, 0.0), (1e-5, 0.0)))
    a = lbm.Sim([lbm.workload_instance(w)])
    b = lbm.Sim([lbm.workload_instance(w)])
    c = lbm.Sim([lbm.workload_instance(w)])
    try:
        def check(n):
            c.step(n)
            assert torch.equal(a.populations(), c.populations())
            b.set_populations(a.populations())
            fa, fb = a.fields(), b.fields()
            assert all(torch.equal(x, y) for x, y in zip(fa, fb))
        a.step(5)
        check(5)
        rho = a.fields()[0].contiguous()
        F = torch.empty((2, 2, 40, 96), dtype=torch.float32, device=rho.device)
        lbm.lbm_forces(a.ctx, 0, rho.data_ptr(), F.data_ptr())
        a.step(3)
        check(3)
        store = torch.empty((3, lbm.lbm_record_floats(a.ctx, 0)), dtype=torch.float32, device=rho.device)
        lbm.lbm_record(a.ctx, 0, 3, store.data_ptr())
        check(3)
        lbm.lbm_set_tiling(a.ctx, 5)
        a.step(16 + 3)  # a graph replay and eager steps
        check(19)
        lbm.lbm_set_balance(a.ctx, 2)
        a.step(7)
        check(7)
        lbm.lbm_set_strip_width(a.ctx, 40)
        lbm.lbm_set_tiling(a.ctx, 2)
        a.step(4)
        check(4)
        lbm.lbm_set_strip_width(a.ctx, 506)
        with pytest.raises(lbm.LBMError):
            lbm.lbm_set_strip_width(a.ctx, 507)
    finally:
        a.close()
        b.close()
        c.close()


def test_batched_balanced_plan_equals_uniform(torch):
    """The 96-instance mix under a balanced plan (shares spanning instances) equals the
    uniform plan bit for bit."""
    say("batched balanced plan")
    ws = W.batched()[:24]
    outs = []
    for bal in (0, 2):
        sim = lbm.Sim([lbm.workload_instance(w) for w in ws])
        lbm.lbm_set_strip_width(sim.ctx, 58)
        if bal:
            lbm.lbm_set_balance(sim.ctx, bal)
        sim.step(17)
        outs.append([sim.populations(i).cpu().numpy() for i in (0, 5, 23)])
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------- velocity-shift forcing
def shift_instance(nx, ny, walls=0, seed=5, tau=(1.0, 0.7)):
    w = W.droplet(nx=nx, ny=ny, radius=min(nx, ny) / 4, couplings=W.COUPLINGS_PAPER, tau=tau)
    d = lbm.workload_instance(w)
    d["forcing"] = lbm.LBM_FORCING_SHIFT
    if walls:
        d.update(walls=1, rho_wall=(0.03, 1.0), g=((1e-5, 0.0), (1e-5, 0.0)))
    return d


def shift_oparams(d):
    return O.Params(nx=d["nx"], ny=d["ny"], G_AB=d["G_AB"], G1=d["G1"], G2=d["G2"], tau=d["tau"],
                    g=d.get("g", ((0.0, 0.0), (0.0, 0.0))), walls=d.get("walls", 0),
                    rho_wall=d.get("rho_wall", (0.0, 0.0)), forcing=1)


@pytest.mark.parametrize("walls", [0, 1])
def test_shift_forcing_single_step(torch, walls):
    """Velocity-shift forcing of the original model: one step from a developed GPU state
    against the oracle's step of the same state."""
    say("shift single step", walls)
    d = shift_instance(70, 37, walls)
    sim = lbm.Sim([d])
    sim.step(30)
    f = sim.populations_full()
    sim.step(1)
    f1 = sim.populations_full()
    want = O.step(shift_oparams(d), f)
    sim.close()
    assert np.abs(f1 - want).max() < 2e-7


def test_shift_forcing_droplet_1000_steps(torch):
    """(equal relaxation times: away from them this droplet diverges under the velocity
    shift, in the oracle as well, the scheme's known instability)"""
    say("shift droplet 1000 steps")
    d = shift_instance(64, 64, tau=(1.0, 1.0))
    sim = lbm.Sim([d])
    sim.step(1000)
    rho, u = sim.fields()
    p = shift_oparams(d)
    flo = O.fields(p, O.run(p, O.init(p, d["rhoA"], d["rhoB"]), 1000))
    er = [rel(rho.cpu().numpy()[k], flo["rho"][k]) for k in range(2)]
    eu = [rel(u.cpu().numpy()[k], flo["u"][k]) for k in range(2)]
    say("errors", er, eu)
    sim.close()
    assert max(er) <= 1e-5 and max(eu) <= 5e-5, (er, eu)


def test_shift_forcing_plans_and_adjoint_refusal(torch):
    say("shift plans")
    d = shift_instance(200, 40)
    ref = None
    for cols, h in ((58, 16), (240, 10), (112, 7), (48, -2)):
        sim = lbm.Sim([d])
        lbm.lbm_set_strip_width(sim.ctx, cols)
        if h > 0:
            lbm.lbm_set_tiling(sim.ctx, h)
        else:
            lbm.lbm_set_balance(sim.ctx, -h)
        sim.step(19)
        f = sim.populations().cpu().numpy()
        if ref is None:
            ref = f
            lam = torch.zeros_like(sim.populations())
            with pytest.raises(lbm.LBMError) as ei:
                sim.adjoint_seed("dp", sim.populations(), lam)
            assert ei.value.code == lbm.LBM_EUNSUPPORTED
        sim.close()
        assert np.array_equal(f, ref), (cols, h)
    # one forcing per context
    with pytest.raises(lbm.LBMError) as ei:
        lbm.Sim([d, dict(d, forcing=lbm.LBM_FORCING_GUO)])
    assert ei.value.code == lbm.LBM_EUNSUPPORTED
