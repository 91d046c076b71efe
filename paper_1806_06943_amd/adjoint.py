"""Gradients of LBM objectives with respect to the model parameters.

theta = (G1, G2, G_AB, tau_A, tau_B): the couplings of Eqs. 8 and 9 (G1 and
G2 move both components together) and the relaxation times of Eq. 1
(arXiv:1806.06943).  An objective J (pressure jump, flow rate, momentum,
mass; see ``lbm.OBJECTIVES``) of the state after a number of steps is
differentiated in reverse mode with checkpoint-and-recompute: the forward
pass keeps the state at the start of each window of steps and records the
states of the last window as it goes; the backward pass re-runs each earlier
window forward from its checkpoint, storing its states, and applies the
library's adjoint step (``lbm_adjoint_step``) backwards through the window.
The re-run of the window before runs meanwhile, in a second library context
on a second stream fed by a second host thread, into the other of two state
stores (events order each store's reuse), so the two latency-bound passes
overlap.
Memory: one state per window boundary plus two windows of states; a run
that is one window (window 0 picks that when every state of the run fits in
the device memory) needs one store and re-runs nothing.

Argument marshalling and bookkeeping only: the step, the adjoint step and the
objective seeds all run in the HIP library.
"""
from __future__ import annotations

import threading

import numpy as np

from . import lbm
from . import trace


class Problem:
    """J(f(steps); theta) for one lattice instance, with its gradient.

    ``instance`` is an instance dict for ``lbm.Sim``; the initial state is the
    equilibrium at rest of its densities (as ``lbm_init`` builds it).
    """

    def __init__(self, instance: dict, steps: int, objective: str, window: int = 200,
                 device: str = "cuda:0", memory_fraction: float = 0.7):
        if steps < 0 or window < 0:
            raise ValueError("steps must be >= 0 and window >= 0 (0: chosen by memory)")
        self.sim = lbm.Sim([instance], device=device)
        self.torch = self.sim.torch
        # the context that re-runs windows, on a stream of its own (default
        # priority), beside the adjoint sweep of the following window
        self.rec = lbm.Sim([instance], device=device,
                           stream=self.torch.cuda.Stream(device=self.sim.device))
        self.steps = int(steps)
        self.objective = objective
        self.f0 = self.sim.populations(0).clone()
        p = self.sim.params[0]
        self.shape = (2, 9, p.ny, p.nx)
        self.nodes = p.nx * p.ny
        self._store = None
        self._forwards = 0
        self._last_intact = False
        self.window = int(window) if window > 0 else self.auto_window(memory_fraction)

    def state_bytes(self) -> int:
        """Bytes of one recorded state (populations and densities)."""
        return 4 * int(lbm.lbm_record_floats(self.rec.ctx, 0))

    def auto_window(self, fraction: float = 0.7) -> int:
        """The whole run as one window when all its states fit in `fraction` of
        the free device memory (one store, no window re-run), else the largest
        window whose two stores fit."""
        per = self.state_bytes()
        t = self.torch
        free, _ = t.cuda.mem_get_info(self.sim.device)
        # memory the caching allocator holds but does not use is free for the store too
        free += t.cuda.memory_reserved(self.sim.device) - t.cuda.memory_allocated(self.sim.device)
        budget = fraction * free
        n = max(self.steps, 1)
        if n * per <= budget:
            return n
        return max(1, min(n, int(budget // (2 * per))))

    def theta(self) -> np.ndarray:
        return self.sim.theta(0)

    def _windows(self):
        out, s = [], 0
        while s < self.steps:
            n = min(self.window, self.steps - s)
            out.append((s, n))
            s += n
        return out

    def _stores(self):
        """The window stores of states, two (one for a run that is one window),
        allocated once for windows of up to `window` steps."""
        m = min(self.window, max(self.steps, 1))
        ns = 1 if len(self._windows()) <= 1 else 2
        if self._store is None or self._store.shape[0] < ns or self._store.shape[1] < m:
            t = self.torch
            self._store = None
            self._store = t.empty((ns, m, lbm.lbm_record_floats(self.rec.ctx, 0)), dtype=t.float32,
                                  device=self.sim.device)
        return self._store

    def forward(self, theta):
        """J at theta; returns (J, saved) where saved feeds ``backward``."""
        t = self.torch
        self.sim.set_theta(theta)
        self.sim.set_populations(self.f0)
        ckpts = []
        wins = self._windows()
        for w, (_, n) in enumerate(wins):
            with trace.range(f"forward window {w}"):
                c = t.empty(self.shape, dtype=t.float32, device=self.sim.device)
                self.sim.populations_into(c)
                ckpts.append(c)
                if w == len(wins) - 1:
                    # the last window's states go straight to the store its adjoint
                    # sweep reads, so the backward pass need not re-run it
                    lbm.lbm_record(self.sim.ctx, 0, n, self._stores()[w % 2].data_ptr())
                else:
                    self.sim.step(n)
        fT = t.empty(self.shape, dtype=t.float32, device=self.sim.device)
        self.sim.populations_into(fT)
        lamT = t.empty(self.shape, dtype=t.float32, device=self.sim.device)
        J, direct = self.sim.adjoint_seed(self.objective, fT, lamT)
        self._forwards += 1  # names the forward pass whose last window the store holds
        self._last_intact = True
        return J, (np.asarray(theta, dtype=np.float64).copy(), ckpts, lamT, direct, self._forwards)

    def backward(self, saved):
        """(dJ/dtheta as numpy float64[5], dJ/df(0) as a device tensor)."""
        t = self.torch
        theta, ckpts, lamT, direct, token = saved
        # the store still holds this forward pass's last window unless another
        # forward pass or the re-runs of an earlier backward pass wrote over it
        last_kept = token == self._forwards and self._last_intact
        self.sim.set_theta(theta)
        S = self._stores()
        grad = t.zeros(5, dtype=t.float64, device=self.sim.device)
        lam = lamT.clone()
        tmp = t.empty_like(lam)
        wins = self._windows()
        rec, adj = self.rec, self.sim
        rec.set_theta(theta)
        # the checkpoints and the seed come from the adjoint context's stream
        rec.stream.wait_stream(adj.stream)
        nw = len(wins)
        # the store of the last window is written over when window nw - 3
        # re-runs into it, or when this pass re-runs its own last window
        # there (its forward pass is not the one whose window the store holds)
        if nw >= 3 or not last_kept:
            self._last_intact = False
        recorded = [t.cuda.Event() for _ in range(nw)]  # window w re-run into S[w % 2]
        released = [t.cuda.Event() for _ in range(nw)]  # sweep of window w done with it
        queued_rec = [threading.Event() for _ in range(nw)]
        queued_adj = [threading.Event() for _ in range(nw)]
        failed = []

        # One host thread per stream: a launch that blocks on a full queue
        # (a long run of launches waiting for the other stream) then holds up
        # only its own stream.  The order between the streams is kept on the
        # GPU by the events; the host events only make sure that an event is
        # recorded before the other thread queues a wait on it.
        def rerun_all():
            try:
                for w in range(nw - 1, -1, -1):
                    if w + 2 < nw:  # S[w % 2] was last read by the sweep of window w + 2
                        queued_adj[w + 2].wait()
                        if failed:
                            return
                        rec.stream.wait_event(released[w + 2])
                    if w < nw - 1 or not last_kept:  # else recorded by the forward pass
                        with trace.range(f"re-run window {w}"):
                            rec.set_populations(ckpts[w])
                            lbm.lbm_record(rec.ctx, 0, wins[w][1], S[w % 2].data_ptr())
                    recorded[w].record(rec.stream)
                    queued_rec[w].set()
            except BaseException as e:  # re-raised by the caller
                failed.append(e)
                for q in queued_rec:
                    q.set()

        th = threading.Thread(target=rerun_all, daemon=True)
        th.start()
        try:
            for w in range(nw - 1, -1, -1):
                queued_rec[w].wait()
                if failed:
                    break
                adj.stream.wait_event(recorded[w])
                with trace.range(f"adjoint window {w}"):
                    lbm.lbm_adjoint_run(adj.ctx, 0, wins[w][1], S[w % 2].data_ptr(),
                                        lam.data_ptr(), tmp.data_ptr(), grad.data_ptr())
                released[w].record(adj.stream)
                queued_adj[w].set()
        except BaseException as e:
            failed.append(e)
        finally:
            for q in queued_adj:
                q.set()
            th.join()
        if failed:
            raise failed[0]
        g = grad.cpu().numpy() + direct
        return g, lam

    def value_and_grad(self, theta=None):
        theta = self.theta() if theta is None else theta
        J, saved = self.forward(theta)
        g, lam0 = self.backward(saved)
        return J, g, lam0

    def close(self):
        self._store = None
        self.rec.close()
        self.sim.close()


def _function():
    import torch

    class LBMObjective(torch.autograd.Function):
        """J(theta) of a Problem as a differentiable torch scalar (float64, CPU)."""

        @staticmethod
        def forward(ctx, theta, problem):
            J, saved = problem.forward(theta.detach().cpu().double().numpy())
            ctx.problem = problem
            ctx.saved = saved
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            g, _ = ctx.problem.backward(ctx.saved)
            ctx.saved = None
            return gJ * torch.from_numpy(g), None

    return LBMObjective


_FN = None


def objective(theta, problem: Problem):
    """Differentiable J(theta): ``theta`` a float64 tensor of 5 values."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(theta, problem)
