"""ctypes wrapper and FP64 observables of the CPU oracle (arXiv:1806.06943).

TEST INFRASTRUCTURE ONLY.  Arrays are float64 numpy arrays in the layouts

* ``f``   ``[2, 9, ny, nx]``  populations, component k (A=0, B=1), direction i
* ``rho`` ``[2, ny, nx]``
* ``F``, ``j`` ``[2, 2, ny, nx]`` (component, axis x/y)
* ``u``   ``[2, ny, nx]``  (axis, y, x)

The step itself is the C code in ``lbm_oracle.c``; the observables below are
plain numpy reductions of the oracle's fields, each citing the passage of the
paper it follows.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_ORACLE_SO selects another build of the same source (the sanitizer test
# loads an address- and undefined-behaviour-sanitized one)
_SO = os.environ.get("LBM_ORACLE_SO") or os.path.join(_HERE, "_lbm_oracle.so")

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


class _CParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("walls", ctypes.c_int),
        ("G_AB", ctypes.c_double), ("G1", ctypes.c_double * 2), ("G2", ctypes.c_double * 2),
        ("tau", ctypes.c_double * 2), ("rho0", ctypes.c_double),
        ("g", ctypes.c_double * 4), ("rho_wall", ctypes.c_double * 2),
        ("forcing", ctypes.c_int),
    ]


@dataclasses.dataclass
class Params:
    """Model parameters as the paper states them (Eqs. 1, 8, 9; Sec. II B)."""
    nx: int
    ny: int
    G_AB: float
    G1: float | tuple = -7.4
    G2: float | tuple = 6.4
    tau: tuple = (1.0, 1.0)
    rho0: float = 1.0
    g: tuple = ((0.0, 0.0), (0.0, 0.0))
    walls: int = 0
    rho_wall: tuple = (0.0, 0.0)
    forcing: int = 0   # 0: Guo term (present model), 1: velocity shift (original model)

    def c(self) -> _CParams:
        def pair(v):
            return (float(v), float(v)) if np.isscalar(v) else (float(v[0]), float(v[1]))
        c = _CParams()
        c.nx, c.ny, c.walls = int(self.nx), int(self.ny), int(self.walls)
        c.G_AB = float(self.G_AB)
        c.G1[:] = pair(self.G1)
        c.G2[:] = pair(self.G2)
        c.tau[:] = pair(self.tau)
        c.rho0 = float(self.rho0)
        gg = np.asarray(self.g, dtype=np.float64).reshape(2, 2)
        c.g[:] = [float(v) for v in gg.ravel()]
        c.rho_wall[:] = pair(self.rho_wall)
        c.forcing = int(self.forcing)
        return c


_lib = None


def lib():
    """Load the oracle shared library, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_CParams)
        L.ora_tables.argtypes = [_I, _I, _I, _D, _I, _I, _D]
        L.ora_density.argtypes = [P, _D, _D]
        L.ora_forces.argtypes = [P, _D, _D]
        L.ora_feq.argtypes = [ctypes.c_double] * 3 + [_D]
        L.ora_guo.argtypes = [ctypes.c_double] * 5 + [_D]
        L.ora_shift.argtypes = [ctypes.c_double] * 6 + [_D]
        L.ora_pressure.argtypes = [P, _D, _D]
        L.ora_step.argtypes = [P, _D, _D, _D]
        L.ora_run.argtypes = [P, _D, ctypes.c_long, _D]
        L.ora_step_at.argtypes = [P, _D, ctypes.c_int, ctypes.c_int, _D]
        L.ora_init.argtypes = [P, _D, _D, _D]
        L.ora_fields.argtypes = [P, _D, _D, _D, _D, _D, _D, _D]
        L.ora_threads.restype = ctypes.c_int
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_adjoint_step.argtypes = [P, _D, _D, _D, _D, _D]
        L.ora_objective.argtypes = [P, _D, ctypes.c_int, _D, _D, _D]
        L.ora_objective.restype = ctypes.c_double
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads used by the oracle's row loops."""
    return int(lib().ora_threads())


def set_threads(n: int):
    """OpenMP threads for the following row loops (timing only)."""
    lib().ora_set_threads(int(n))


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


# ---------------------------------------------------------------- tables
def tables():
    """Return the oracle's lattice tables: (ex9, ey9, opp9, w9, ex25, ey25, p25)."""
    ex9 = (ctypes.c_int * 9)(); ey9 = (ctypes.c_int * 9)(); opp = (ctypes.c_int * 9)()
    w9 = (ctypes.c_double * 9)()
    ex25 = (ctypes.c_int * 25)(); ey25 = (ctypes.c_int * 25)(); p25 = (ctypes.c_double * 25)()
    lib().ora_tables(ex9, ey9, opp, w9, ex25, ey25, p25)
    return (list(ex9), list(ey9), list(opp), list(w9), list(ex25), list(ey25), list(p25))


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().ora_feq(rho, ux, uy, _ptr(out))
    return out


def guo(tau, ux, uy, Fx, Fy):
    out = np.zeros(9)
    lib().ora_guo(tau, ux, uy, Fx, Fy, _ptr(out))
    return out


def shift(tau, rho, ux, uy, Fx, Fy):
    """Velocity-shift forcing term C^SC of the original model (Sec. II A)."""
    out = np.zeros(9)
    lib().ora_shift(tau, rho, ux, uy, Fx, Fy, _ptr(out))
    return out


# ---------------------------------------------------------------- lattice calls
def init(p: Params, rhoA: np.ndarray, rhoB: np.ndarray) -> np.ndarray:
    """Equilibrium at rest, f_{k,i} = w_i rho_k (reading of the unstated initialisation)."""
    rhoA = np.ascontiguousarray(rhoA, dtype=np.float64)
    rhoB = np.ascontiguousarray(rhoB, dtype=np.float64)
    assert rhoA.shape == (p.ny, p.nx) and rhoB.shape == (p.ny, p.nx)
    f = np.zeros((2, 9, p.ny, p.nx))
    c = p.c()
    lib().ora_init(ctypes.byref(c), _ptr(rhoA), _ptr(rhoB), _ptr(f))
    return f


def density(p: Params, f: np.ndarray) -> np.ndarray:
    rho = np.zeros((2, p.ny, p.nx))
    c = p.c()
    lib().ora_density(ctypes.byref(c), _ptr(np.ascontiguousarray(f)), _ptr(rho))
    return rho


def forces(p: Params, rho: np.ndarray) -> np.ndarray:
    """Total force F_k = F^c_k + F^r_k + F^b_k from a density field (Eqs. 8, 9)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    assert rho.shape == (2, p.ny, p.nx)
    F = np.zeros((2, 2, p.ny, p.nx))
    c = p.c()
    lib().ora_forces(ctypes.byref(c), _ptr(rho), _ptr(F))
    return F


def step(p: Params, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    work = np.zeros((4, p.ny, p.nx))
    c = p.c()
    lib().ora_step(ctypes.byref(c), _ptr(f), _ptr(out), _ptr(work))
    return out


def run(p: Params, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Return f advanced by nsteps (the input array is not modified)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    work = np.zeros((22, p.ny, p.nx))
    c = p.c()
    lib().ora_run(ctypes.byref(c), _ptr(f), int(nsteps), _ptr(work))
    return f


def step_at(p: Params, f: np.ndarray, x: int, y: int) -> np.ndarray:
    """Next-step populations [2, 9] at node (x, y), touching only its neighbourhood."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(18)
    c = p.c()
    lib().ora_step_at(ctypes.byref(c), _ptr(f), int(x), int(y), _ptr(out))
    return out.reshape(2, 9)


def fields(p: Params, f: np.ndarray) -> dict:
    """rho, j (with F/2), F, u^eq, barycentric u and bulk pressure p_b."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    sh = (p.ny, p.nx)
    out = dict(rho=np.zeros((2,) + sh), j=np.zeros((2, 2) + sh), F=np.zeros((2, 2) + sh),
               ueq=np.zeros((2,) + sh), u=np.zeros((2,) + sh), pb=np.zeros(sh))
    c = p.c()
    lib().ora_fields(ctypes.byref(c), _ptr(f), _ptr(out["rho"]), _ptr(out["j"]),
                     _ptr(out["F"]), _ptr(out["ueq"]), _ptr(out["u"]), _ptr(out["pb"]))
    return out


# ---------------------------------------------------------------- adjoint (FP64)
THETA_NAMES = ("G1", "G2", "G_AB", "tau_A", "tau_B")
OBJECTIVES = {"dp": 0, "Q": 1, "momA": 2, "mom": 3, "massA": 4}


def with_theta(p: Params, theta) -> Params:
    """p with theta = (G1, G2, G_AB, tau_A, tau_B); G1, G2 set for both components."""
    t = [float(v) for v in theta]
    return dataclasses.replace(p, G1=(t[0], t[0]), G2=(t[1], t[1]), G_AB=t[2], tau=(t[3], t[4]))


def theta_of(p: Params) -> np.ndarray:
    def first(v):
        return float(v) if np.isscalar(v) else float(v[0])
    return np.array([first(p.G1), first(p.G2), float(p.G_AB), float(p.tau[0]), float(p.tau[1])])


def adjoint_step(p: Params, f: np.ndarray, lam_next: np.ndarray):
    """(dPhi/df)^T lam_next and (dPhi/dtheta)^T lam_next for one step from state f."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    lam = np.zeros_like(f)
    grad = np.zeros(5)
    work = np.zeros((10, p.ny, p.nx))
    c = p.c()
    lib().ora_adjoint_step(ctypes.byref(c), _ptr(f), _ptr(lam_next), _ptr(lam), _ptr(grad),
                           _ptr(work))
    return lam, grad


def objective(p: Params, f: np.ndarray, which: str | int):
    """(J, dJ/df, direct dJ/dtheta) of a differentiable observable of state f."""
    w = OBJECTIVES[which] if isinstance(which, str) else int(which)
    f = np.ascontiguousarray(f, dtype=np.float64)
    lam = np.zeros_like(f)
    dth = np.zeros(5)
    work = np.zeros((10, p.ny, p.nx))
    c = p.c()
    J = lib().ora_objective(ctypes.byref(c), _ptr(f), w, _ptr(lam), _ptr(dth), _ptr(work))
    return float(J), lam, dth


def value_and_grad(p: Params, f0: np.ndarray, steps: int, which: str | int):
    """J(f(steps)) and its gradients with respect to theta and f0.

    Stores every intermediate state (small lattices only) and runs the
    adjoint steps backwards from the objective's seed.
    """
    states = [np.ascontiguousarray(f0, dtype=np.float64)]
    for _ in range(steps):
        states.append(step(p, states[-1]))
    J, lam, g = objective(p, states[-1], which)
    g = g.copy()
    for t in range(steps - 1, -1, -1):
        lam, gs = adjoint_step(p, states[t], lam)
        g += gs
    return J, g, lam


def objective_after(p: Params, f0: np.ndarray, steps: int, which: str | int) -> float:
    """J(f(steps)) only (for finite differences)."""
    return objective(p, run(p, f0, steps), which)[0]


# ---------------------------------------------------------------- pressure tensor (FP64)
def pressure(p: Params, f: np.ndarray) -> np.ndarray:
    """P[c][y][x], c = xx, yy, xy: pair-sum interaction part plus kinetic part (Sec. II B)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    P = np.zeros((3, p.ny, p.nx))
    c = p.c()
    lib().ora_pressure(ctypes.byref(c), _ptr(f), _ptr(P))
    return P


def line_tension(P: np.ndarray) -> float:
    """Eq. 15 / Eq. 16 for interfaces orthogonal to x: sum_x (P_xx - P_yy), mean over y."""
    return float((P[0] - P[1]).sum(axis=1).mean())


def disjoining_pressure(h: np.ndarray, gf: np.ndarray, gamma: float) -> np.ndarray:
    """Eq. 18 from gamma_f(h) on a grid of h: s = gamma_f - 2 gamma,
    Pi(h) = s(h)/h - int_h^inf s/h'^2 dh' (trapezoid rule, s beyond the last h taken as 0)."""
    h = np.asarray(h, dtype=np.float64)
    s = np.asarray(gf, dtype=np.float64) - 2.0 * gamma
    g = s / h ** 2
    tail = np.zeros_like(h)
    for j in range(len(h) - 2, -1, -1):
        tail[j] = tail[j + 1] + 0.5 * (g[j] + g[j + 1]) * (h[j + 1] - h[j])
    return s / h - tail


# ---------------------------------------------------------------- observables (numpy, FP64)
E9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])


def masses(f: np.ndarray) -> np.ndarray:
    """Per-component mass M_k = sum_x rho_k (Eq. 6)."""
    return f.sum(axis=(1, 2, 3))


def raw_momentum(f: np.ndarray) -> np.ndarray:
    """Total population momentum P = sum_{x,k,i} f_{k,i} e_i (no force shift)."""
    s = f.sum(axis=(2, 3))  # [k, i]
    return np.array([(s * E9[:, 0]).sum(), (s * E9[:, 1]).sum()])


def laplace(p: Params, fl: dict, out_margin: float = 12.0) -> dict:
    """Static-droplet pressure jump and surface tension (Laplace test, Sec. III B).

    The paper does not state its protocol; the reading used here:
    rho_in/out = max/min of rho_A; droplet area A = sum (rho_A - out)/(in - out),
    R_eff = sqrt(A/pi); centre = periodic circular mean of (rho_A - out);
    <p>_in over nodes with r <= R_eff/2, <p>_out over r >= R_eff + out_margin
    (minimum-image distance); gamma = (<p>_in - <p>_out) R_eff in 2-D.
    """
    rA = fl["rho"][0]
    pb = fl["pb"]
    ny, nx = rA.shape
    rin, rout = rA.max(), rA.min()
    wgt = rA - rout
    area = wgt.sum() / (rin - rout)
    R = math.sqrt(area / math.pi)
    xs = np.arange(nx)
    ys = np.arange(ny)
    wx = wgt.sum(axis=0)
    wy = wgt.sum(axis=1)
    cx = (math.atan2((wx * np.sin(2 * np.pi * xs / nx)).sum(),
                     (wx * np.cos(2 * np.pi * xs / nx)).sum()) * nx / (2 * np.pi)) % nx
    cy = (math.atan2((wy * np.sin(2 * np.pi * ys / ny)).sum(),
                     (wy * np.cos(2 * np.pi * ys / ny)).sum()) * ny / (2 * np.pi)) % ny
    dx = np.abs(xs[None, :] - cx)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(ys[:, None] - cy)
    dy = np.minimum(dy, ny - dy)
    r = np.sqrt(dx * dx + dy * dy)
    inside = r <= R / 2
    outside = r >= R + out_margin
    p_in = pb[inside].mean()
    p_out = pb[outside].mean()
    return dict(R=R, cx=cx, cy=cy, p_in=p_in, p_out=p_out, dp=p_in - p_out,
                gamma=(p_in - p_out) * R, n_in=int(inside.sum()), n_out=int(outside.sum()))


def interface_width_row(row: np.ndarray, start: int) -> float:
    """Interface width W = (rho_max - rho_min) / (rho(M) - rho(N)) (Fig. 2 caption).

    M and N are the two adjacent nodes straddling rho_bar = (max + min)/2,
    found by walking in +x (periodically) from ``start`` inside the droplet.
    """
    n = row.shape[0]
    rmax, rmin = row.max(), row.min()
    bar = 0.5 * (rmax + rmin)
    x = start
    for _ in range(n):
        xn = (x + 1) % n
        if row[x] >= bar > row[xn]:
            return float((rmax - rmin) / (row[x] - row[xn]))
        x = xn
    return float("nan")


def width_from_values(rho_max, rho_min, rho_M, rho_N) -> float:
    """The same formula on four given numbers."""
    return (rho_max - rho_min) / (rho_M - rho_N)


def flow_profile(fl: dict) -> np.ndarray:
    """u_bar(y): x-average of the barycentric x velocity (Sec. III D)."""
    return fl["u"][0].mean(axis=1)


def flow_rate(fl: dict) -> float:
    """Q = sum_y u_bar(y) (Sec. III D, the integral over the channel with dy = 1)."""
    return float(flow_profile(fl).sum())


def max_speed(fl: dict) -> float:
    """Maximum |u| of the barycentric velocity (Appendix, spurious currents)."""
    u = fl["u"]
    return float(np.sqrt(u[0] ** 2 + u[1] ** 2).max())


def radial_correlation(phi: np.ndarray, rmax: int | None = None):
    """Radially averaged two-point correlation of a periodic field:
    C(r) = <phi(x) phi(x + d)>_{x, |d| in [r - 1/2, r + 1/2)} - <phi>^2, normalised
    by C(0) (Wiener-Khinchin: the autocorrelation by FFT, a library step)."""
    phi = np.asarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    d = phi - phi.mean()
    ac = np.fft.ifft2(np.abs(np.fft.fft2(d)) ** 2).real / d.size
    dy = np.minimum(np.arange(ny), ny - np.arange(ny))[:, None]
    dx = np.minimum(np.arange(nx), nx - np.arange(nx))[None, :]
    rbin = np.rint(np.sqrt(dx * dx + dy * dy)).astype(int)
    rmax = min(nx, ny) // 2 if rmax is None else rmax
    sums = np.bincount(rbin.ravel(), weights=ac.ravel(), minlength=rmax + 1)[:rmax + 1]
    counts = np.bincount(rbin.ravel(), minlength=rmax + 1)[:rmax + 1]
    C = sums / np.maximum(counts, 1)
    return C / C[0]


def domain_size(phi: np.ndarray) -> float:
    """Mean domain size of a demixing pattern: the first zero of the radial
    correlation of phi, linearly interpolated between lattice distances."""
    C = radial_correlation(phi)
    for r in range(1, len(C)):
        if C[r] <= 0.0 < C[r - 1]:
            return float(r - 1 + C[r - 1] / (C[r - 1] - C[r]))
    return float("nan")
