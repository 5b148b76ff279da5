"""Plain PyTorch float64 CPU statement of the base step, for gradients.

TEST INFRASTRUCTURE ONLY.  The reference for the adjoint is the definition of
a vector-Jacobian product: torch.autograd applied to this straightforward
re-statement of the maps of GENGA II Sect. 2 (kick of eq. Hb with the
changeover of Sect. 6.2, HC of eq. Hc, Kepler drift of eq. Ha, critical radii
of eq. rcrit) in the order of Appendix A.  It is independent of the HIP
library and of the C oracle (whose forward values it is checked against).

Shapes: positions and velocities are (N, 3) tensors, masses and critical radii
(N,).  Everything is O(N^2) in memory: meant for N up to a few hundred.
"""
from __future__ import annotations

import torch

TD = torch.float64


def changeover(y: torch.Tensor) -> torch.Tensor:
    """K(y) of Chambers (1999) eq. 10 on y = (r - 0.1 rho) / (0.9 rho)."""
    mid = y * y / (2.0 * y * y - 2.0 * y + 1.0)
    return torch.where(y <= 0.0, torch.zeros_like(y), torch.where(y >= 1.0, torch.ones_like(y), mid))


def pair_rho(rc: torch.Tensor) -> torch.Tensor:
    """rho_ij = max(rc_i, rc_j); on a tie the lower index owns the value."""
    n = rc.shape[0]
    ri, rj = rc[:, None].expand(n, n), rc[None, :].expand(n, n)
    idx = torch.arange(n)
    tie = torch.where(idx[:, None] < idx[None, :], ri, rj)
    return torch.where(ri > rj, ri, torch.where(ri < rj, rj, tie))


def kick_acc(x: torch.Tensor, m: torch.Tensor, rc: torch.Tensor, G: float) -> torch.Tensor:
    """a_i = G sum_{j != i} m_j K(r_ij; rho_ij) (x_j - x_i) / r_ij^3."""
    n = x.shape[0]
    d = x[None, :, :] - x[:, None, :]               # d[i, j] = x_j - x_i
    eye = torch.eye(n, dtype=torch.bool)
    r2 = (d * d).sum(-1)
    r2s = torch.where(eye, torch.ones_like(r2), r2)
    r = torch.sqrt(r2s)
    rho = pair_rho(rc)
    K = changeover((r - 0.1 * rho) / (0.9 * rho))
    w = torch.where(eye, torch.zeros_like(r2), G * K / (r2s * r))
    return ((w * m[None, :])[:, :, None] * d).sum(1)


def rcrit(x, v, m, m_star, dt, n1, n2):
    """r_crit = max(n1 R_H, n2 |dt| |v|), R_H = |x| (m / 3 m_star)^(1/3); ties -> Hill term."""
    a = n1 * torch.linalg.norm(x, dim=1) * (m / (3.0 * m_star)) ** (1.0 / 3.0)
    b = n2 * abs(dt) * torch.linalg.norm(v, dim=1)
    return torch.where(a >= b, a, b)


def hc(x, v, m, m_star, h):
    """x += h P / m_star, P = sum m v."""
    P = (m[:, None] * v).sum(0)
    return x + h * P[None, :] / m_star


def _drift_bound(x, v, r0, u, alpha, mu, dt, iters):
    """Gauss f and g in the eccentric-anomaly change dE (alpha = 1/a > 0).
    Kepler's equation n dt = dE - ec sin dE + es (1 - cos dE), ec = 1 - r0/a,
    es = u / sqrt(mu a), is solved without gradient tracking; one more Newton
    step taken with tracking gives the derivative of the exact root
    (implicit-function theorem)."""
    a = 1.0 / alpha
    n = torch.sqrt(mu * alpha ** 3)
    ec = 1.0 - r0 * alpha
    es = u / torch.sqrt(mu * a)
    M = n * dt

    def F(d):
        return d - ec * torch.sin(d) + es * (1.0 - torch.cos(d)) - M

    def Fp(d):
        return 1.0 - ec * torch.cos(d) + es * torch.sin(d)

    with torch.no_grad():
        d = M.clone()
        for _ in range(iters):
            d = d - F(d) / Fp(d)
    d = d.detach()
    d = d - F(d) / Fp(d)
    s, c = torch.sin(d), torch.cos(d)
    omc = 2.0 * torch.sin(0.5 * d) ** 2
    r = a + (r0 - a) * c + torch.sqrt(a) * (u / mu ** 0.5) * s
    f = 1.0 - (a / r0) * omc
    g = dt - (d - s) / n
    fd = -torch.sqrt(mu * a) * s / (r * r0)
    gd = 1.0 - (a / r) * omc
    return f[:, None] * x + g[:, None] * v, fd[:, None] * x + gd[:, None] * v


def _drift_unbound(x, v, r0, u, alpha, mu, dt, iters):
    """Gauss f and g in the hyperbolic-anomaly change dF (alpha = 1/a < 0,
    A = -a > 0).  With e cosh F0 = 1 + r0/A and e sinh F0 = u / sqrt(mu A),
    the mean-anomaly change e sinh F - F gives Kepler's equation
    n dt = ch sinh dF + sh (cosh dF - 1) - dF, n = sqrt(mu / A^3), and
    r = A (ch cosh dF + sh sinh dF - 1); f = 1 - (A/r0)(cosh dF - 1),
    g = dt - (sinh dF - dF)/n, fdot = -sqrt(mu A) sinh dF / (r r0),
    gdot = 1 - (A/r)(cosh dF - 1).  Root as in the bound case."""
    A = -1.0 / alpha
    n = torch.sqrt(mu / A ** 3)
    ch = 1.0 + r0 / A
    sh = u / torch.sqrt(mu * A)
    M = n * dt

    def F(d):
        return ch * torch.sinh(d) + sh * (torch.cosh(d) - 1.0) - d - M

    def Fp(d):
        return ch * torch.cosh(d) + sh * torch.sinh(d) - 1.0

    with torch.no_grad():
        d = torch.asinh(M / ch)
        for _ in range(iters):
            d = d - F(d) / Fp(d)
    d = d.detach()
    d = d - F(d) / Fp(d)
    s, c = torch.sinh(d), torch.cosh(d)
    cm1 = 2.0 * torch.sinh(0.5 * d) ** 2
    r = A * (ch * c + sh * s - 1.0)
    f = 1.0 - (A / r0) * cm1
    g = dt - (s - d) / n
    fd = -torch.sqrt(mu * A) * s / (r * r0)
    gd = 1.0 - (A / r) * cm1
    return f[:, None] * x + g[:, None] * v, fd[:, None] * x + gd[:, None] * v


def drift(x, v, mu, dt, iters: int = 60):
    """Kepler drift about mu for dt by Gauss f and g: bound orbits in the
    eccentric-anomaly change, unbound ones in the hyperbolic-anomaly change
    (each body takes its own branch; a parabolic orbit, 1/a = 0, is refused)."""
    r0 = torch.linalg.norm(x, dim=1)
    v2 = (v * v).sum(1)
    u = (x * v).sum(1)
    alpha = 2.0 / r0 - v2 / mu
    bound = alpha > 0
    if bool((alpha == 0).any()):
        raise ValueError("torch reference drift: parabolic orbit")
    if bool(bound.all()):
        return _drift_bound(x, v, r0, u, alpha, mu, dt, iters)
    ib = torch.nonzero(bound).flatten()
    iu = torch.nonzero(~bound).flatten()
    xo = torch.zeros_like(x)
    vo = torch.zeros_like(v)
    for idx, fn in ((ib, _drift_bound), (iu, _drift_unbound)):
        if idx.numel() == 0:
            continue
        xs, vs = fn(x[idx], v[idx], r0[idx], u[idx], alpha[idx], mu, dt, iters)
        xo = xo.index_copy(0, idx, xs)
        vo = vo.index_copy(0, idx, vs)
    return xo, vo


def step(x, v, m, G, m_star, dt, n1, n2):
    """One base step (Appendix A without the direct solver)."""
    h = 0.5 * dt
    rc = rcrit(x, v, m, m_star, dt, n1, n2)
    v = v + h * kick_acc(x, m, rc, G)
    x = hc(x, v, m, m_star, h)
    x, v = drift(x, v, G * m_star, dt)
    x = hc(x, v, m, m_star, h)
    v = v + h * kick_acc(x, m, rc, G)
    return x, v


def simulate(x, v, m, steps, G, m_star, dt, n1, n2):
    for _ in range(steps):
        x, v = step(x, v, m, G, m_star, dt, n1, n2)
    return x, v


def state_tensors(d: dict, requires_grad: bool = False):
    """(x (N,3), v (N,3), m (N,)) float64 tensors from a workload dict."""
    import numpy as np
    x = torch.tensor(np.stack([d["x"], d["y"], d["z"]]), dtype=TD).T.contiguous()
    v = torch.tensor(np.stack([d["vx"], d["vy"], d["vz"]]), dtype=TD).T.contiguous()
    m = torch.tensor(d["m"], dtype=TD)
    if requires_grad:
        x.requires_grad_(True)
        v.requires_grad_(True)
        m.requires_grad_(True)
    return x, v, m
