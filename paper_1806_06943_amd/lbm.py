"""Python binding of the HIP library ``liblbm_hip.so`` (C-ABI in include/lbm.h).

Argument marshalling only: every function below forwards to the C entry point
of the same name; all lattice arithmetic runs in the library's HIP kernels.
PyTorch supplies device memory (the workspace and the field buffers) and the
stream.  There is no CPU fallback: if the library is missing or fails to load,
every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# LBM_HIP_SO selects another build of the same sources (the sanitizer test
# loads one whose host code is address- and undefined-behaviour-sanitized)
LIB_PATH = os.environ.get("LBM_HIP_SO") or os.path.join(_PKG, "liblbm_hip.so")

LBM_OK = 0
LBM_EINVAL = -1
LBM_EHIP = -2
LBM_ENONFINITE = -3
LBM_EUNSUPPORTED = -4

# objectives of lbm_adjoint_seed
LBM_OBJ_DP = 0
LBM_OBJ_Q = 1
LBM_OBJ_MOM_A = 2
LBM_OBJ_MOM = 3
LBM_OBJ_MASS_A = 4
OBJECTIVES = {"dp": LBM_OBJ_DP, "Q": LBM_OBJ_Q, "momA": LBM_OBJ_MOM_A, "mom": LBM_OBJ_MOM,
              "massA": LBM_OBJ_MASS_A}
THETA_NAMES = ("G1", "G2", "G_AB", "tau_A", "tau_B")


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("forcing", ctypes.c_int32),
        ("G_AB", ctypes.c_double), ("G1", ctypes.c_double * 2), ("G2", ctypes.c_double * 2),
        ("tau", ctypes.c_double * 2), ("psi_rho0", ctypes.c_double),
        ("g", (ctypes.c_double * 2) * 2), ("rho_wall", ctypes.c_double * 2),
        ("rho_ref", ctypes.c_double * 2),
    ]


class lbm_obs(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double * 2), ("mom_raw", ctypes.c_double * 2),
        ("mom_bary", ctypes.c_double * 2), ("max_speed", ctypes.c_double),
        ("rho_a_max", ctypes.c_double), ("rho_a_min", ctypes.c_double),
        ("flow_rate", ctypes.c_double), ("R_eff", ctypes.c_double),
        ("cx", ctypes.c_double), ("cy", ctypes.c_double),
        ("p_in", ctypes.c_double), ("p_out", ctypes.c_double), ("dp", ctypes.c_double),
        ("gamma", ctypes.c_double), ("width", ctypes.c_double),
        ("n_in", ctypes.c_int64), ("n_out", ctypes.c_int64), ("finite", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblbm_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.lbm_workspace_bytes.argtypes = [P(lbm_params), ctypes.c_int32, P(ctypes.c_uint64)]
        L.lbm_init.argtypes = [P(vp), P(lbm_params), ctypes.c_int32, P(ctypes.c_double),
                               P(ctypes.c_double), vp, ctypes.c_uint64, vp]
        L.lbm_step.argtypes = [vp, ctypes.c_int64]
        L.lbm_prepare.argtypes = [vp]
        L.lbm_steps_done.argtypes = [vp]
        L.lbm_steps_done.restype = ctypes.c_int64
        L.lbm_observables.argtypes = [vp, P(lbm_obs), P(ctypes.c_double)]
        L.lbm_observables_noalloc.argtypes = [vp, P(lbm_obs)]
        L.lbm_fields.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.lbm_get_populations.argtypes = [vp, ctypes.c_int32, vp]
        L.lbm_set_populations.argtypes = [vp, ctypes.c_int32, vp]
        L.lbm_forces.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.lbm_copy_probe.argtypes = [vp, vp, vp, ctypes.c_uint64]
        L.lbm_profile_step.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double),
                                       P(ctypes.c_char_p), P(ctypes.c_int32)]
        L.lbm_set_tiling.argtypes = [vp, ctypes.c_int32]
        L.lbm_get_tiling.argtypes = [vp]
        L.lbm_get_tiling.restype = ctypes.c_int32
        L.lbm_set_strip_width.argtypes = [vp, ctypes.c_int32]
        L.lbm_set_balance.argtypes = [vp, ctypes.c_int32]
        L.lbm_get_balance.argtypes = [vp]
        L.lbm_get_balance.restype = ctypes.c_int32
        L.lbm_plan_workgroups.argtypes = [P(lbm_params), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          P(ctypes.c_int32), P(ctypes.c_int32)]
        L.lbm_set_full_rows.argtypes = [vp, ctypes.c_int32]
        L.lbm_get_full_rows.argtypes = [vp]
        L.lbm_get_full_rows.restype = ctypes.c_int32
        L.lbm_set_two_step.argtypes = [vp, ctypes.c_int32]
        L.lbm_get_two_step.argtypes = [vp]
        L.lbm_get_two_step.restype = ctypes.c_int32
        L.lbm_get_workgroups.argtypes = [vp]
        L.lbm_get_workgroups.restype = ctypes.c_int32
        L.lbm_get_strip_width.argtypes = [vp]
        L.lbm_get_strip_width.restype = ctypes.c_int32
        L.lbm_adjoint_step.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp]
        L.lbm_adjoint_seed.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                       P(ctypes.c_double), P(ctypes.c_double)]
        L.lbm_set_params.argtypes = [vp, ctypes.c_int32, P(lbm_params)]
        L.lbm_record.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp]
        L.lbm_record_floats.argtypes = [vp, ctypes.c_int32]
        L.lbm_record_floats.restype = ctypes.c_int64
        L.lbm_pressure.argtypes = [vp, ctypes.c_int32, vp, P(ctypes.c_double)]
        L.lbm_adjoint_run.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp]
        L.lbm_profile_adjoint.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32,
                                          ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_char_p),
                                          P(ctypes.c_int32)]
        L.lbm_lds_checks.argtypes = [vp, P(ctypes.c_int64)]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, ctx=None):
    if rc != LBM_OK:
        msg = lib().lbm_last_error(ctx)
        raise LBMError(rc, msg.decode() if msg else "")


LBM_FORCING_GUO = 0
LBM_FORCING_SHIFT = 1


def make_params(nx, ny, G_AB, G1, G2, tau, g=((0.0, 0.0), (0.0, 0.0)), walls=0,
                rho_wall=(0.0, 0.0), rho_ref=(0.0, 0.0), psi_rho0=1.0,
                forcing=LBM_FORCING_GUO) -> lbm_params:
    def pair(v):
        return (float(v), float(v)) if np.isscalar(v) else (float(v[0]), float(v[1]))
    p = lbm_params()
    p.nx, p.ny, p.walls, p.forcing = int(nx), int(ny), int(walls), int(forcing)
    p.G_AB = float(G_AB)
    p.G1[:] = pair(G1)
    p.G2[:] = pair(G2)
    p.tau[:] = pair(tau)
    p.psi_rho0 = float(psi_rho0)
    gg = np.asarray(g, dtype=np.float64).reshape(2, 2)
    for k in range(2):
        p.g[k][0], p.g[k][1] = float(gg[k, 0]), float(gg[k, 1])
    p.rho_wall[:] = pair(rho_wall)
    # the library works with the FP32 value of the reference; keep it exact
    p.rho_ref[:] = tuple(float(np.float32(v)) for v in pair(rho_ref))
    return p


# ------------------------------------------------------------- C entry points, same names
def lbm_workspace_bytes(params) -> int:
    arr = (lbm_params * len(params))(*params)
    out = ctypes.c_uint64()
    _check(lib().lbm_workspace_bytes(arr, len(params), ctypes.byref(out)))
    return int(out.value)


def lbm_init(params, rhoA0: np.ndarray, rhoB0: np.ndarray, workspace_ptr: int,
             workspace_bytes: int, stream_ptr: int):
    arr = (lbm_params * len(params))(*params)
    a = np.ascontiguousarray(rhoA0, dtype=np.float64)
    b = np.ascontiguousarray(rhoB0, dtype=np.float64)
    ctx = ctypes.c_void_p()
    rc = lib().lbm_init(ctypes.byref(ctx), arr, len(params),
                        a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        ctypes.c_void_p(workspace_ptr), workspace_bytes, ctypes.c_void_p(stream_ptr))
    _check(rc, None)
    return ctx


def lbm_step(ctx, nsteps: int):
    _check(lib().lbm_step(ctx, int(nsteps)), ctx)


def lbm_prepare(ctx):
    _check(lib().lbm_prepare(ctx), ctx)


def lbm_steps_done(ctx) -> int:
    return int(lib().lbm_steps_done(ctx))


def lbm_observables(ctx, n_inst: int, total_rows: int | None = None, check: bool = True):
    out = (lbm_obs * n_inst)()
    ubar = None
    up = None
    if total_rows:
        ubar = np.zeros(total_rows)
        up = ubar.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = lib().lbm_observables(ctx, out, up)
    if check or rc not in (LBM_OK, LBM_ENONFINITE):
        _check(rc, ctx)
    return rc, [o.as_dict() for o in out], ubar


def lbm_observables_noalloc(ctx, n_inst: int, check: bool = True):
    out = (lbm_obs * n_inst)()
    rc = lib().lbm_observables_noalloc(ctx, out)
    if check or rc not in (LBM_OK, LBM_ENONFINITE):
        _check(rc, ctx)
    return rc, [o.as_dict() for o in out]


def lbm_fields(ctx, inst: int, rho_ptr: int | None, u_ptr: int | None):
    _check(lib().lbm_fields(ctx, inst, ctypes.c_void_p(rho_ptr), ctypes.c_void_p(u_ptr)), ctx)


def lbm_get_populations(ctx, inst: int, f_ptr: int):
    _check(lib().lbm_get_populations(ctx, inst, ctypes.c_void_p(f_ptr)), ctx)


def lbm_set_populations(ctx, inst: int, f_ptr: int):
    _check(lib().lbm_set_populations(ctx, inst, ctypes.c_void_p(f_ptr)), ctx)


def lbm_forces(ctx, inst: int, rho_ptr: int, F_ptr: int):
    _check(lib().lbm_forces(ctx, inst, ctypes.c_void_p(rho_ptr), ctypes.c_void_p(F_ptr)), ctx)


def lbm_copy_probe(ctx, dst_ptr: int, src_ptr: int, nbytes: int):
    _check(lib().lbm_copy_probe(ctx, ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nbytes)), ctx)


def lbm_profile_step(ctx, nrep: int, max_k: int = 8):
    ms = (ctypes.c_double * max_k)()
    names = (ctypes.c_char_p * max_k)()
    nk = ctypes.c_int32()
    _check(lib().lbm_profile_step(ctx, int(nrep), max_k, ms, names, ctypes.byref(nk)), ctx)
    n = min(nk.value, max_k)
    return [(names[j].decode(), ms[j]) for j in range(n)]


def lbm_set_tiling(ctx, chunk_rows: int):
    _check(lib().lbm_set_tiling(ctx, int(chunk_rows)), ctx)


def lbm_get_tiling(ctx) -> int:
    return int(lib().lbm_get_tiling(ctx))


def lbm_set_strip_width(ctx, cols: int):
    _check(lib().lbm_set_strip_width(ctx, int(cols)), ctx)


def lbm_get_strip_width(ctx) -> int:
    return int(lib().lbm_get_strip_width(ctx))


def lbm_set_balance(ctx, wgs_per_cu: int):
    _check(lib().lbm_set_balance(ctx, int(wgs_per_cu)), ctx)


def lbm_get_balance(ctx) -> int:
    return int(lib().lbm_get_balance(ctx))


def lbm_plan_workgroups(params, cols: int, chunk_rows: int = 16, wgs: int = 0,
                        full_rows: int = 0):
    """(workgroups, segments) of a strip plan, planned on the host."""
    arr = (lbm_params * len(params))(*params)
    nwg, nseg = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbm_plan_workgroups(arr, len(params), int(cols), int(chunk_rows), int(wgs),
                                     int(full_rows), ctypes.byref(nwg), ctypes.byref(nseg)))
    return int(nwg.value), int(nseg.value)


def lbm_set_full_rows(ctx, on: int):
    _check(lib().lbm_set_full_rows(ctx, int(on)), ctx)


def lbm_get_full_rows(ctx) -> int:
    return int(lib().lbm_get_full_rows(ctx))


def lbm_set_two_step(ctx, on: int):
    _check(lib().lbm_set_two_step(ctx, int(on)), ctx)


def lbm_get_two_step(ctx) -> int:
    return int(lib().lbm_get_two_step(ctx))


def lbm_get_workgroups(ctx) -> int:
    return int(lib().lbm_get_workgroups(ctx))


def lbm_adjoint_step(ctx, inst: int, f_ptr: int, lam_in_ptr: int, lam_out_ptr: int,
                     grad_ptr: int | None):
    _check(lib().lbm_adjoint_step(ctx, inst, ctypes.c_void_p(f_ptr), ctypes.c_void_p(lam_in_ptr),
                                  ctypes.c_void_p(lam_out_ptr), ctypes.c_void_p(grad_ptr)), ctx)


def lbm_adjoint_seed(ctx, inst: int, objective: int, f_ptr: int, lam_ptr: int | None):
    """(J, direct dJ/dtheta as a numpy array of 5)."""
    J = ctypes.c_double()
    dth = (ctypes.c_double * 5)()
    _check(lib().lbm_adjoint_seed(ctx, inst, int(objective), ctypes.c_void_p(f_ptr),
                                  ctypes.c_void_p(lam_ptr), ctypes.byref(J), dth), ctx)
    return float(J.value), np.array(list(dth))


def lbm_pressure(ctx, inst: int, P_ptr: int, want_line_tension: bool = True):
    """Pressure tensor into P_ptr ([3][ny][nx] FP32); returns the line tension or None."""
    lt = ctypes.c_double()
    _check(lib().lbm_pressure(ctx, inst, ctypes.c_void_p(P_ptr),
                              ctypes.byref(lt) if want_line_tension else None), ctx)
    return float(lt.value) if want_line_tension else None


def lbm_record_floats(ctx, inst: int) -> int:
    n = int(lib().lbm_record_floats(ctx, inst))
    if n < 0:
        raise LBMError(LBM_EINVAL, "bad context or instance")
    return n


def lbm_record(ctx, inst: int, nsteps: int, f_store_ptr: int):
    _check(lib().lbm_record(ctx, inst, int(nsteps), ctypes.c_void_p(f_store_ptr)), ctx)


def lbm_adjoint_run(ctx, inst: int, nsteps: int, f_store_ptr: int, lam_ptr: int, tmp_ptr: int,
                    grad_ptr: int | None):
    _check(lib().lbm_adjoint_run(ctx, inst, int(nsteps), ctypes.c_void_p(f_store_ptr),
                                 ctypes.c_void_p(lam_ptr), ctypes.c_void_p(tmp_ptr),
                                 ctypes.c_void_p(grad_ptr)), ctx)


def lbm_set_params(ctx, inst: int, params: lbm_params):
    _check(lib().lbm_set_params(ctx, inst, ctypes.byref(params)), ctx)


def lbm_profile_adjoint(ctx, inst: int, f_ptr: int, lam_in_ptr: int, lam_out_ptr: int,
                        grad_ptr: int, nrep: int, max_k: int = 8):
    ms = (ctypes.c_double * max_k)()
    names = (ctypes.c_char_p * max_k)()
    nk = ctypes.c_int32()
    _check(lib().lbm_profile_adjoint(ctx, inst, ctypes.c_void_p(f_ptr), ctypes.c_void_p(lam_in_ptr),
                                     ctypes.c_void_p(lam_out_ptr), ctypes.c_void_p(grad_ptr),
                                     int(nrep), max_k, ms, names, ctypes.byref(nk)), ctx)
    n = min(nk.value, max_k)
    return [(names[j].decode(), ms[j]) for j in range(n)]


def lbm_lds_checks(ctx) -> int:
    """Out-of-range LDS indices seen since the last call (checked build only)."""
    n = ctypes.c_int64()
    _check(lib().lbm_lds_checks(ctx, ctypes.byref(n)), ctx)
    return int(n.value)


def lbm_destroy(ctx):
    _check(lib().lbm_destroy(ctx), None)


# ------------------------------------------------------------- torch-owned memory wrapper
class Sim:
    """One context over one or more instances, with its workspace in a torch tensor.

    ``instances`` is a list of dicts with keys nx, ny, rhoA, rhoB, G_AB, G1, G2,
    tau and optionally g, walls, rho_wall, forcing, rho_ref (default: the mean
    initial density of each component, the reference of the FP32 deviation
    storage).
    """

    def __init__(self, instances, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = []
        rA, rB = [], []
        for w in instances:
            rho_ref = w.get("rho_ref")
            if rho_ref is None:
                rho_ref = (float(np.mean(w["rhoA"])), float(np.mean(w["rhoB"])))
            self.params.append(make_params(w["nx"], w["ny"], w["G_AB"], w["G1"], w["G2"], w["tau"],
                                           g=w.get("g", ((0.0, 0.0), (0.0, 0.0))),
                                           walls=w.get("walls", 0),
                                           rho_wall=w.get("rho_wall", (0.0, 0.0)),
                                           rho_ref=rho_ref,
                                           forcing=w.get("forcing", LBM_FORCING_GUO)))
            rA.append(np.asarray(w["rhoA"], dtype=np.float64).ravel())
            rB.append(np.asarray(w["rhoB"], dtype=np.float64).ravel())
        self.n_inst = len(self.params)
        self.ws_bytes = lbm_workspace_bytes(self.params)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            # int64 elements keep the base 256-byte aligned (allocator granularity)
            self.workspace = torch.empty((self.ws_bytes + 7) // 8, dtype=torch.int64, device=self.device)
            self.ctx = lbm_init(self.params, np.concatenate(rA), np.concatenate(rB),
                                self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream)
        self.total_rows = sum(p.ny for p in self.params)

    # --------------------------------------------------------------- stepping
    def step(self, n: int = 1):
        lbm_step(self.ctx, n)

    def prepare(self):
        """Capture the step graphs of both state parities now (see lbm_prepare)."""
        lbm_prepare(self.ctx)

    @property
    def steps_done(self) -> int:
        return lbm_steps_done(self.ctx)

    def observables(self, check: bool = True):
        rc, obs, ubar = lbm_observables(self.ctx, self.n_inst, self.total_rows, check=check)
        self.last_rc = rc
        return obs, ubar

    # --------------------------------------------------------------- fields
    def fields(self, inst: int = 0):
        p = self.params[inst]
        t = self.torch
        rho = t.empty((2, p.ny, p.nx), dtype=t.float32, device=self.device)
        u = t.empty((2, p.ny, p.nx), dtype=t.float32, device=self.device)
        lbm_fields(self.ctx, inst, rho.data_ptr(), u.data_ptr())
        self.stream.synchronize()
        return rho, u

    def populations(self, inst: int = 0):
        """FP32 deviations f - w_i rho_ref, [2, 9, ny, nx] on the device."""
        p = self.params[inst]
        f = self.torch.empty((2, 9, p.ny, p.nx), dtype=self.torch.float32, device=self.device)
        lbm_get_populations(self.ctx, inst, f.data_ptr())
        self.stream.synchronize()
        return f

    def populations_full(self, inst: int = 0) -> np.ndarray:
        """f itself in float64 (deviation plus w_i rho_ref), [2, 9, ny, nx] on the host."""
        p = self.params[inst]
        f = self.populations(inst).cpu().numpy().astype(np.float64)
        w = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1], dtype=np.float64) / 36.0
        return f + w[None, :, None, None] * np.asarray(p.rho_ref[:])[:, None, None, None]

    def pressure(self, inst: int = 0):
        """(P [3, ny, nx] FP32 on the device, line tension sum (P_xx - P_yy) / ny)."""
        p = self.params[inst]
        P = self.torch.empty((3, p.ny, p.nx), dtype=self.torch.float32, device=self.device)
        lt = lbm_pressure(self.ctx, inst, P.data_ptr())
        return P, lt

    def populations_into(self, f_dev, inst: int = 0):
        """Export the populations into a contiguous [2, 9, ny, nx] FP32 device tensor (async)."""
        assert f_dev.is_contiguous() and f_dev.dtype == self.torch.float32
        lbm_get_populations(self.ctx, inst, f_dev.data_ptr())

    def set_populations(self, f_dev, inst: int = 0):
        lbm_set_populations(self.ctx, inst, f_dev.data_ptr())

    # --------------------------------------------------------------- parameters and adjoint
    def theta(self, inst: int = 0) -> np.ndarray:
        """theta = (G1, G2, G_AB, tau_A, tau_B) of an instance (component A's G1, G2)."""
        p = self.params[inst]
        return np.array([p.G1[0], p.G2[0], p.G_AB, p.tau[0], p.tau[1]], dtype=np.float64)

    def set_theta(self, theta, inst: int = 0):
        """Set G1, G2 (both components), G_AB, tau_A, tau_B of an instance."""
        t = [float(v) for v in theta]
        p = lbm_params.from_buffer_copy(self.params[inst])
        p.G1[:] = (t[0], t[0])
        p.G2[:] = (t[1], t[1])
        p.G_AB = t[2]
        p.tau[:] = (t[3], t[4])
        lbm_set_params(self.ctx, inst, p)
        self.params[inst] = p

    def adjoint_step(self, f_dev, lam_in, lam_out, grad_dev=None, inst: int = 0):
        """lam_out = (df(t+1)/df(t))^T lam_in at state f_dev; grad_dev += theta part (async)."""
        lbm_adjoint_step(self.ctx, inst, f_dev.data_ptr(), lam_in.data_ptr(), lam_out.data_ptr(),
                         None if grad_dev is None else grad_dev.data_ptr())

    def adjoint_seed(self, objective, f_dev, lam_dev=None, inst: int = 0):
        """(J, direct dJ/dtheta) of state f_dev; lam_dev receives dJ/df."""
        obj = OBJECTIVES[objective] if isinstance(objective, str) else int(objective)
        return lbm_adjoint_seed(self.ctx, inst, obj, f_dev.data_ptr(),
                                None if lam_dev is None else lam_dev.data_ptr())

    def forces(self, rho_dev, inst: int = 0):
        p = self.params[inst]
        F = self.torch.empty((2, 2, p.ny, p.nx), dtype=self.torch.float32, device=self.device)
        lbm_forces(self.ctx, inst, rho_dev.contiguous().data_ptr(), F.data_ptr())
        self.stream.synchronize()
        return F

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workload_instance(w, rho_ref=None) -> dict:
    """Instance dict for Sim from a workloads.Workload."""
    d = dict(nx=w.nx, ny=w.ny, rhoA=w.rhoA, rhoB=w.rhoB, G_AB=w.G_AB, G1=w.G1, G2=w.G2,
             tau=w.tau, g=w.g, walls=w.walls, rho_wall=w.rho_wall)
    if rho_ref is not None:
        d["rho_ref"] = rho_ref
    return d
