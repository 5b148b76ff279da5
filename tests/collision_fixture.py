"""Two small bodies on a collision course near 1 AU (not a test module):
body 0 on a circular orbit, body 1 a little behind it along the orbit and
catching up, both with radius R.  The reference for one base step with the
direct solver: the K-weighted kick and the Sun kick of the oracle (pinned
elsewhere), and between them the direct solver's flow integrated by scipy's
DOP853 up to the contact r = R_0 + R_1 located by its event finder, the
merger by the formulas of the paper, and the merged body's Kepler flow to the
end of the step."""
import numpy as np
from scipy.integrate import solve_ivp

import oracle
from paper_2201_10058_amd import workload as W

G = W.GAUSS_G


def two_bodies(m0=1e-9, m1=1e-9, R=1e-5, gap=1e-4, dv=1e-4, offset=0.0):
    """offset: radial offset of body 1 (an impact parameter)."""
    v = np.sqrt(G / 1.0)
    st = {"x": np.array([1.0, 1.0 + offset]), "y": np.array([0.0, -gap]), "z": np.array([0.0, 0.0]),
          "vx": np.array([0.0, 0.0]), "vy": np.array([v, v + dv]), "vz": np.array([0.0, 0.0]),
          "m": np.array([m0, m1]), "R": np.array([R, R])}
    return st


def reference_step(st, dt, n1=3.0, n2=0.4):
    s = {k: np.array(v, dtype=np.float64) for k, v in st.items()}
    rc = oracle.rcrit(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], 1.0, dt, n1, n2)
    oracle.kick(s, rc, G, 0.5 * dt)
    oracle.hc(s, 1.0, 0.5 * dt)
    m = s["m"].copy()

    def K(r, rho):
        return oracle.changeover(r, rho)

    rho = max(rc[0], rc[1])

    def f(t, u):
        X, V = u[:6].reshape(2, 3), u[6:].reshape(2, 3)
        A = -G * X / np.linalg.norm(X, axis=1)[:, None] ** 3
        d = X[1] - X[0]
        r = np.linalg.norm(d)
        w = G * (1.0 - K(r, rho)) * d / r ** 3
        A[0] += m[1] * w
        A[1] -= m[0] * w
        return np.concatenate([V.ravel(), A.ravel()])

    def contact(t, u):
        return np.linalg.norm(u[3:6] - u[0:3]) - (s["R"][0] + s["R"][1])
    contact.terminal = True
    contact.direction = -1
    u0 = np.concatenate([np.stack([s["x"], s["y"], s["z"]], 1).ravel(),
                         np.stack([s["vx"], s["vy"], s["vz"]], 1).ravel()])
    sol = solve_ivp(f, (0, dt), u0, method="DOP853", rtol=1e-13, atol=1e-18, events=contact)
    assert sol.status == 1, "no contact within the step"
    tc = sol.t_events[0][0]
    u = sol.y_events[0][0]
    X, V = u[:6].reshape(2, 3), u[6:].reshape(2, 3)
    M = m[0] + m[1]
    xm = (m[0] * X[0] + m[1] * X[1]) / M
    vm = (m[0] * V[0] + m[1] * V[1]) / M
    dU = 0.5 * m[0] * m[1] / M * np.sum((V[0] - V[1]) ** 2) - G * m[0] * m[1] / np.linalg.norm(X[0] - X[1])
    surv, gone = (0, 1) if (m[0] > m[1] or (m[0] == m[1])) else (1, 0)

    def kep(t, u):
        return np.concatenate([u[3:], -G * u[:3] / np.linalg.norm(u[:3]) ** 3])
    sol2 = solve_ivp(kep, (tc, dt), np.concatenate([xm, vm]), method="DOP853", rtol=1e-13,
                     atol=1e-18)
    y = sol2.y[:, -1]
    out = {k: v.copy() for k, v in s.items()}
    for c, k in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        out[k][surv] = y[c]
    out["x"][gone], out["y"][gone], out["z"][gone] = 1e6 + gone, 0.0, 0.0
    out["vx"][gone] = out["vy"][gone] = out["vz"][gone] = 0.0
    out["m"][surv], out["m"][gone] = M, 0.0
    out["R"][surv] = np.cbrt(s["R"][0] ** 3 + s["R"][1] ** 3)
    out["R"][gone] = 0.0
    oracle.hc(out, 1.0, 0.5 * dt)
    oracle.kick(out, rc, G, 0.5 * dt)
    return out, tc, (surv, gone, dU)
