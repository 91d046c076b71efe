"""Seeded synthetic workloads (initial density fields and parameter sets).

This module holds geometry and random numbers only: discs, noise, rejection
sampling of droplet centres.  It contains none of the lattice Boltzmann
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

Every field is float64 ``[ny, nx]`` and is generated once on the host by
``numpy.random.Generator(PCG64(SEED_BASE + workload_index))``.

The paper runs on synthetic geometries only (a static droplet, a channel
emulsion, planar films); these generators stand in for them at the sizes the
benchmarks use:

* ``droplet``  64x64 torus, one disc of A (R=12) in B, noise +-1e-3
* ``spinodal`` 2048x2048 torus, rho_A = 0.5 + U(-0.05, 0.05), rho_B = 1 - rho_A
* ``emulsion`` 4096x512 channel, 200 discs of A (R=16) in B between walls
* ``batched``  96 droplet instances, sides {64,128,192,256}, seeded radii/G_2
* ``adjoint``  512x512 torus, 16 discs of R=20
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 1806069430

# (G_AB, G_1, G_2) couplings.  The literal set of the droplet workload does not
# demix (uniform mixture is linearly stable); the set used in the paper's
# emulsion section (gamma = 0.04) does.
COUPLINGS_LITERAL = (0.405, -9.0, 8.1)
COUPLINGS_PAPER = (3.0, -7.4, 6.4)

RHO_DENSE = 1.0    # majority-component density inside its own phase
RHO_DILUTE = 0.03  # minority-component density


def rng(index: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index + 1000 * sub))


def disc_fields(nx: int, ny: int, centres, radius, inside=(RHO_DENSE, RHO_DILUTE),
                outside=(RHO_DILUTE, RHO_DENSE), periodic_y: bool = True):
    """Sharp discs of phase A (densities ``inside``) in phase B (``outside``).

    ``radius`` may be a scalar or one value per centre.  Distances use the
    minimum image in x, and in y when ``periodic_y``.
    """
    xs = np.arange(nx)[None, :]
    ys = np.arange(ny)[:, None]
    mask = np.zeros((ny, nx), dtype=bool)
    radii = np.broadcast_to(np.asarray(radius, dtype=np.float64), (len(centres),))
    for (cx, cy), r in zip(centres, radii):
        dx = np.abs(xs - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(ys - cy)
        if periodic_y:
            dy = np.minimum(dy, ny - dy)
        mask |= (dx * dx + dy * dy) <= r * r
    rhoA = np.where(mask, inside[0], outside[0]).astype(np.float64)
    rhoB = np.where(mask, inside[1], outside[1]).astype(np.float64)
    return rhoA, rhoB


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    rhoA: np.ndarray
    rhoB: np.ndarray
    G_AB: float
    G1: float
    G2: float
    tau: tuple
    g: tuple = ((0.0, 0.0), (0.0, 0.0))
    walls: int = 0
    rho_wall: tuple = (0.0, 0.0)
    steps: int = 0
    extra: dict = dataclasses.field(default_factory=dict)


def droplet(nx: int = 64, ny: int = 64, radius: float = 12.0, noise: float = 1e-3,
            couplings=COUPLINGS_LITERAL, tau=(1.0, 0.6), index: int = 0, sub: int = 0,
            steps: int = 1000) -> Workload:
    """Static droplet: a disc of A at the centre of a periodic box, seeded noise."""
    r = rng(index, sub)
    rhoA, rhoB = disc_fields(nx, ny, [(nx // 2, ny // 2)], radius)
    rhoA = rhoA + r.uniform(-noise, noise, size=(ny, nx))
    rhoB = rhoB + r.uniform(-noise, noise, size=(ny, nx))
    G_AB, G1, G2 = couplings
    return Workload("droplet", nx, ny, rhoA, rhoB, G_AB, G1, G2, tuple(tau), steps=steps,
                    extra=dict(radius=radius))


def spinodal(nx: int = 2048, ny: int = 2048, couplings=COUPLINGS_LITERAL,
             tau=(1.0, 0.55), index: int = 1, steps: int = 20000) -> Workload:
    """Spinodal decomposition: rho_A = 0.5 + U(-0.05, 0.05) per node, rho_B = 1 - rho_A."""
    r = rng(index)
    rhoA = 0.5 + r.uniform(-0.05, 0.05, size=(ny, nx))
    rhoB = 1.0 - rhoA
    G_AB, G1, G2 = couplings
    return Workload("spinodal", nx, ny, rhoA, rhoB, G_AB, G1, G2, tuple(tau), steps=steps)


def _place_discs(r: np.random.Generator, nx: int, ny: int, n: int, radius: float,
                 gap: float, ymargin: float, periodic_y: bool, max_tries: int = 200000):
    """Rejection sampling of n centres with pairwise spacing >= 2R + gap."""
    centres = []
    dmin = 2 * radius + gap
    tries = 0
    while len(centres) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could not place {n} discs of radius {radius} in {nx}x{ny}")
        cx = r.uniform(0, nx)
        cy = r.uniform(ymargin, ny - ymargin) if not periodic_y else r.uniform(0, ny)
        ok = True
        for (px, py) in centres:
            dx = abs(cx - px)
            dx = min(dx, nx - dx)
            dy = abs(cy - py)
            if periodic_y:
                dy = min(dy, ny - dy)
            if dx * dx + dy * dy < dmin * dmin:
                ok = False
                break
        if ok:
            centres.append((cx, cy))
    return centres


def emulsion(nx: int = 4096, ny: int = 512, ndrop: int = 200, radius: float = 16.0,
             tau_ratio: float = 1.0, gx: float = 1e-6, index: int = 2,
             steps: int = 50000) -> Workload:
    """Pressure-driven emulsion: discs of A in B between two walls, body force along x.

    The viscosity ratio is read as nu_A / nu_B = tau_ratio with tau_B = 1.0,
    i.e. tau_A = 0.5 + 0.5 * tau_ratio.
    """
    r = rng(index)
    if ndrop > 0:
        centres = _place_discs(r, nx, ny, ndrop, radius, 8.0, radius + 6.0, periodic_y=False)
        rhoA, rhoB = disc_fields(nx, ny, centres, radius, periodic_y=False)
    else:
        centres = []
        rhoA = np.full((ny, nx), RHO_DILUTE)
        rhoB = np.full((ny, nx), RHO_DENSE)
    G_AB, G1, G2 = COUPLINGS_PAPER
    tau = (0.5 + 0.5 * tau_ratio, 1.0)
    return Workload("emulsion", nx, ny, rhoA, rhoB, G_AB, G1, G2, tau,
                    g=((gx, 0.0), (gx, 0.0)), walls=1, rho_wall=(RHO_DILUTE, RHO_DENSE),
                    steps=steps, extra=dict(centres=centres, radius=radius))


def batched(n_inst: int = 96, sizes=(64, 128, 192, 256), index: int = 3,
            steps: int = 5000, noise: float = 1e-3):
    """Uneven static-droplet instances for the batched form.

    Equal numbers of each side length in a seeded order; radius
    ~ U_int[8, min(40, N/2 - 8)]; G_2 ~ U[7.0, 8.5], G_1 = -1 - G_2; G_AB = 3.0;
    tau_B = 1.0 and tau_A cycling over {0.6, 1.0, 1.6}.
    """
    r = rng(index)
    per = n_inst // len(sizes)
    sides = np.repeat(np.asarray(sizes), per)
    sides = np.concatenate([sides, np.full(n_inst - len(sides), sizes[-1])])
    r.shuffle(sides)
    taus = (0.6, 1.0, 1.6)
    out = []
    for n, N in enumerate(sides):
        N = int(N)
        R = int(r.integers(8, min(40, N // 2 - 8) + 1))
        G2 = float(r.uniform(7.0, 8.5))
        rhoA, rhoB = disc_fields(N, N, [(N // 2, N // 2)], R)
        rhoA = rhoA + r.uniform(-noise, noise, size=(N, N))
        rhoB = rhoB + r.uniform(-noise, noise, size=(N, N))
        out.append(Workload(f"batched[{n}]", N, N, rhoA, rhoB, 3.0, -1.0 - G2, G2,
                            (taus[n % 3], 1.0), steps=steps, extra=dict(radius=R)))
    return out


def adjoint_array(nx: int = 512, ny: int = 512, ndrop: int = 16, radius: float = 20.0,
                  gx: float = 1e-6, index: int = 4, steps: int = 4000) -> Workload:
    """Droplet array for gradient calibration: seeded discs, body force along x."""
    r = rng(index)
    centres = _place_discs(r, nx, ny, ndrop, radius, 8.0, 0.0, periodic_y=True)
    rhoA, rhoB = disc_fields(nx, ny, centres, radius)
    G_AB, G1, G2 = COUPLINGS_PAPER
    return Workload("adjoint", nx, ny, rhoA, rhoB, G_AB, G1, G2, (1.0, 0.6),
                    g=((gx, 0.0), (gx, 0.0)), steps=steps, extra=dict(centres=centres))
