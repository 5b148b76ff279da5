"""Gradients of final states with respect to initial positions, velocities and
masses, through trajectories of base steps (Appendix A of GENGA II, without
the direct solver), by the hand-written VJPs of libgenga.so.

The forward pass keeps a checkpoint of (x, v) every `checkpoint_every` steps.
The backward pass recomputes each segment from its checkpoint with the same
kernels (bitwise identical to the forward: every kernel is deterministic),
keeps the per-step intermediate states and applies the adjoints of the
operators in reverse order:

    rc = Rcrit(x0, v0, m)            -> rcrit_vjp
    v1 = v0 + h a(x0, m, rc)         -> kick_vjp(scale = h)
    xa = x0 + h P(v1, m) / m_star     -> hc_vjp
    (xb, v2) = Kepler(xa, v1; dt)    -> drift_vjp
    xc = xb + h P(v2, m) / m_star     -> hc_vjp
    v3 = v2 + h a(xc, m, rc)         -> kick_vjp(scale = h)
"""
from __future__ import annotations

import torch

from . import native as N

_XYZ = ("x", "y", "z")
_V = ("vx", "vy", "vz")


def _state(X, V, m, rc) -> N.State:
    return N.State({"x": X[0], "y": X[1], "z": X[2], "vx": V[0], "vy": V[1], "vz": V[2],
                    "m": m, "rc": rc})


class _Runner:
    def __init__(self, n, cfg: N.Config, device):
        if cfg.c_light or cfg.slevels > 1 or cfg.direct or cfg.tp_mode:
            # the adjoint covers the base step's operators only
            raise N.GengaError(N.E_UNSUPPORTED, "adjoint of a step with GR, levels, the direct "
                               "solver or test particles")
        self.cfg = N.Config(**{**cfg.__dict__, "flags": N.FLAG_NOSYNC, "events": (None,) * 4})
        self.ws = N.Workspace(n, self.cfg, device=device)
        self.h = 0.5 * cfg.dt

    def step_saving(self, X, V, m, rc):
        """One step in place on (X, V); returns the intermediates the adjoint needs."""
        st = _state(X, V, m, rc)
        cfg, ws, h = self.cfg, self.ws, self.h
        x0, v0 = X.clone(), V.clone()
        N.rcrit(st, cfg, ws)
        rc_used = rc.clone()
        N.kick(st, cfg, ws, h)
        v1 = V.clone()
        N.hc(st, cfg, ws, h)
        xa = X.clone()
        N.drift(st, cfg, ws, cfg.dt)
        v2 = V.clone()
        N.hc(st, cfg, ws, h)
        xc = X.clone()
        N.kick(st, cfg, ws, h)
        return dict(x0=x0, v0=v0, rc=rc_used, v1=v1, xa=xa, v2=v2, xc=xc)

    def step(self, X, V, m, rc):
        st = _state(X, V, m, rc)
        code = N.step(st, self.cfg, self.ws)
        if code not in (N.OK,):
            raise N.GengaError(code, "genga_step")

    def step_adjoint(self, sv, m, adj: N.AdjointState):
        """Reverse one step: adj holds (xbar, vbar) of the step's output on entry
        and of its input on exit; adj.m accumulates."""
        cfg, ws, h = self.cfg, self.ws, self.h
        adj.t["rc"].zero_()
        # second half kick at (xc, m, rc): abar = h vbar
        st = _state(sv["xc"], sv["v2"], m, sv["rc"])
        vb = [adj.t[k].clone() for k in _V]
        N.kick_vjp(st, cfg, ws, h, vb, adj)
        # HC at v2
        N.hc_vjp(_state(sv["xc"], sv["v2"], m, sv["rc"]), cfg, ws, h, adj)
        # drift at its input (xa, v1)
        N.drift_vjp(_state(sv["xa"], sv["v1"], m, sv["rc"]), cfg, ws, cfg.dt, adj)
        # HC at v1
        N.hc_vjp(_state(sv["xa"], sv["v1"], m, sv["rc"]), cfg, ws, h, adj)
        # first half kick at (x0, m, rc)
        vb = [adj.t[k].clone() for k in _V]
        N.kick_vjp(_state(sv["x0"], sv["v1"], m, sv["rc"]), cfg, ws, h, vb, adj)
        # critical radii at (x0, v0, m)
        N.rcrit_vjp(_state(sv["x0"], sv["v0"], m, sv["rc"]), cfg, ws, adj)


class Trajectory(torch.autograd.Function):
    """(X0, V0, m) -> (X_T, V_T) after `steps` base steps.  X, V: (3, N)."""

    @staticmethod
    def forward(ctx, X0, V0, m, steps: int, cfg: N.Config, checkpoint_every: int = 20):
        device = X0.device
        n = X0.shape[1]
        run = _Runner(n, cfg, device)
        X = X0.detach().clone().contiguous()
        V = V0.detach().clone().contiguous()
        mm = m.detach().contiguous()
        rc = torch.zeros(n, dtype=torch.float64, device=device)
        ckpts = []
        for k in range(steps):
            if k % checkpoint_every == 0:
                ckpts.append((k, X.clone(), V.clone()))
            run.step(X, V, mm, rc)
        code = N.read_status(run.ws)
        if code != N.OK:
            raise N.GengaError(code, "trajectory forward")
        ctx.save_for_backward(mm)
        ctx.ckpts = ckpts
        ctx.steps = steps
        ctx.cfg = cfg
        ctx.ce = checkpoint_every
        return X, V

    @staticmethod
    def backward(ctx, gX, gV):
        (m,) = ctx.saved_tensors
        n = m.shape[0]
        device = m.device
        run = _Runner(n, ctx.cfg, device)
        adj = N.AdjointState(n, device)
        gX = torch.zeros((3, n), dtype=torch.float64, device=device) if gX is None else gX
        gV = torch.zeros((3, n), dtype=torch.float64, device=device) if gV is None else gV
        for c, k in enumerate(_XYZ):
            adj.t[k].copy_(gX[c])
        for c, k in enumerate(_V):
            adj.t[k].copy_(gV[c])
        rc = torch.zeros(n, dtype=torch.float64, device=device)
        for (k0, Xc, Vc) in reversed(ctx.ckpts):
            k1 = min(k0 + ctx.ce, ctx.steps)
            X, V = Xc.clone(), Vc.clone()
            saved = [run.step_saving(X, V, m, rc) for _ in range(k0, k1)]
            for sv in reversed(saved):
                run.step_adjoint(sv, m, adj)
        code = N.read_status(run.ws)
        if code != N.OK:
            raise N.GengaError(code, "trajectory backward")
        gX0 = torch.stack([adj.t[k] for k in _XYZ])
        gV0 = torch.stack([adj.t[k] for k in _V])
        return gX0, gV0, adj.t["m"].clone(), None, None, None


def simulate(X0, V0, m, steps: int, cfg: N.Config, checkpoint_every: int = 20):
    """Differentiable trajectory: returns (X_T, V_T); gradients flow to X0, V0, m."""
    return Trajectory.apply(X0, V0, m, steps, cfg, checkpoint_every)
