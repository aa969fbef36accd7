"""FP64 reference propagation — TEST INFRASTRUCTURE ONLY.

Plain classical RK4 for the two-body + SRP equations of motion (Sec. 3 of the
paper: y = [x; v], y' = [v; a_g + a_SRP]), with the SRP force from the oracle's
ray tracer at every stage, and the paper's panel update steps 2-4 (Sec. 4.4.2:
panel normal, rotate it as close as possible to the Sun, clamp to the
interval) written out independently of the library.

Readings: the Sun is at the origin and the attitude inertially fixed (Sec. 5.1),
so the Sun direction of a stage is -r/|r|; the pressure scales as
p_ref (r_ref/|r|)^2; a wing root is a panel node whose parent is not a panel;
a panel is two-sided, so of the two angles that face it to the Sun the one of
smaller magnitude is taken, then clamped.
"""
from __future__ import annotations

import numpy as np

from .core import eval_srp, node_transforms


def rk4(f, y0, t0, h, n):
    """Classical RK4 with fixed step h; returns (n+1, 1+len(y0)) rows (t, y)."""
    y = np.array(y0, dtype=np.float64)
    out = np.zeros((n + 1, 1 + y.size))
    out[0, 0], out[0, 1:] = t0, y
    t = t0
    for k in range(n):
        k1 = f(t, y)
        k2 = f(t + h / 2, y + h / 2 * k1)
        k3 = f(t + h / 2, y + h / 2 * k2)
        k4 = f(t + h, y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t = t0 + (k + 1) * h
        out[k + 1, 0], out[k + 1, 1:] = t, y
    return out


# Fehlberg's embedded Runge-Kutta 7(8) pair (13 stages; E. Fehlberg, NASA
# TR R-287, 1968): nodes C, coefficients A (row i uses stages 0..i-1), the
# 8th-order weights B8 and the local error estimate of the 7th-order solution,
# ERR_W (k0 + k10 - k11 - k12) h with ERR_W = 41/840.
F = np.float64
C78 = [F(0), F(2) / 27, F(1) / 9, F(1) / 6, F(5) / 12, F(1) / 2, F(5) / 6, F(1) / 6, F(2) / 3, F(1) / 3, F(1), F(0), F(1)]
A78 = [
    [],
    [F(2) / 27],
    [F(1) / 36, F(1) / 12],
    [F(1) / 24, F(0), F(1) / 8],
    [F(5) / 12, F(0), F(-25) / 16, F(25) / 16],
    [F(1) / 20, F(0), F(0), F(1) / 4, F(1) / 5],
    [F(-25) / 108, F(0), F(0), F(125) / 108, F(-65) / 27, F(125) / 54],
    [F(31) / 300, F(0), F(0), F(0), F(61) / 225, F(-2) / 9, F(13) / 900],
    [F(2), F(0), F(0), F(-53) / 6, F(704) / 45, F(-107) / 9, F(67) / 90, F(3)],
    [F(-91) / 108, F(0), F(0), F(23) / 108, F(-976) / 135, F(311) / 54, F(-19) / 60, F(17) / 6, F(-1) / 12],
    [F(2383) / 4100, F(0), F(0), F(-341) / 164, F(4496) / 1025, F(-301) / 82, F(2133) / 4100, F(45) / 82,
     F(45) / 164, F(18) / 41],
    [F(3) / 205, F(0), F(0), F(0), F(0), F(-6) / 41, F(-3) / 205, F(-3) / 41, F(3) / 41, F(6) / 41, F(0)],
    [F(-1777) / 4100, F(0), F(0), F(-341) / 164, F(4496) / 1025, F(-289) / 82, F(2193) / 4100, F(51) / 82,
     F(33) / 164, F(12) / 41, F(0), F(1)],
]
B78 = [F(0), F(0), F(0), F(0), F(0), F(34) / 105, F(9) / 35, F(9) / 35, F(9) / 280, F(9) / 280, F(0),
       F(41) / 840, F(41) / 840]
ERR_W = F(41) / 840


def rk78_step(f, t, y, h):
    """One step of the 8th-order solution; returns (y_new, error estimate)."""
    k = []
    for i in range(13):
        yi = y.copy()
        for j, a in enumerate(A78[i]):
            if a != 0:
                yi = yi + h * a * k[j]
        k.append(f(t + C78[i] * h, yi))
    y8 = y.copy()
    for i in range(13):
        if B78[i] != 0:
            y8 = y8 + h * B78[i] * k[i]
    err = ERR_W * h * (k[0] + k[10] - k[11] - k[12])
    return y8, err


def rk78(f, y0, t0, t1, h0, rtol=0.0, atol=None, adaptive=False, max_rows=1 << 20):
    """RK7(8) from t0 to t1.  Fixed: n = ceil((t1 - t0)/h0) steps starting at
    t0 + k h0, the last one ending at t1.  Adaptive (adaptive=True): a step is
    accepted when its error estimate satisfies
    max_i |err_i| / (atol_i + rtol max(|y_i|, |y_new_i|)) <= 1 (a component
    with zero error counts 0); the next trial
    step is the step times 0.9 err^(-1/8) clamped to [0.2, 5] (5 when the
    estimate is 0), and a step that would pass t1 is shortened to end there.
    Returns rows (t, y) of the accepted steps (the first row is t0) and the
    number of derivative evaluations."""
    y = np.array(y0, dtype=np.float64)
    atol = np.zeros_like(y) if atol is None else np.broadcast_to(np.asarray(atol, np.float64), y.shape)
    rows = [np.concatenate([[t0], y])]
    evals = 0
    if not adaptive:
        n = max(1, int(np.ceil((t1 - t0) / h0 * (1 - 1e-12))))
        for k in range(n):
            tk = t0 + k * h0
            hs = t1 - tk if k == n - 1 else h0
            y, _ = rk78_step(f, tk, y, hs)
            evals += 13
            rows.append(np.concatenate([[t1 if k == n - 1 else t0 + (k + 1) * h0], y]))
        return np.array(rows), evals
    t, h = t0, h0
    while t < t1:
        last = h >= t1 - t
        hs = t1 - t if last else h
        yn, err = rk78_step(f, t, y, hs)
        evals += 13
        sc = atol + rtol * np.maximum(np.abs(y), np.abs(yn))
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(err == 0, 0.0, np.abs(err) / sc)    # a zero error counts 0 even where sc = 0
        e = np.max(ratio)
        fac = 5.0 if e == 0 else min(5.0, max(0.2, 0.9 * e ** (-1.0 / 8.0)))
        if e > 1.0:
            h = hs * fac
            continue
        t = t1 if last else t + hs
        y = yn
        h = hs * fac
        rows.append(np.concatenate([[t], y]))
        if len(rows) > max_rows:
            raise ValueError("too many steps")
    return np.array(rows), evals


def _rest_normal(mesh, node):
    sel = mesh.tri_node == node
    V = mesh.verts[mesh.tris[sel]]
    n = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]).sum(0)
    return n / np.linalg.norm(n)


def _rot(a, th):
    a = np.asarray(a, float) / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def sun_tracking(mesh, sun_dir, angles):
    """Wing-root angles that turn each root's rest normal towards the Sun."""
    ang = np.array(angles, dtype=np.float64)
    s = np.asarray(sun_dir, float) / np.linalg.norm(sun_dir)
    offs = np.concatenate([[0], np.cumsum(mesh.n_axes)])[:-1]
    for k in range(1, mesh.n_nodes):
        p = mesh.parent[k]
        if not (mesh.is_panel[k] and not mesh.is_panel[p] and mesh.n_axes[k] > 0):
            continue
        Rp = node_transforms(mesh, ang)[p][:, :3]     # parent world rotation (clamped angles)
        sp = Rp.T @ s
        n0 = _rest_normal(mesh, k)
        m_axes = mesh.n_axes[k]
        for a in range(m_axes):
            m = n0.copy()
            for b in range(m_axes - 1, a, -1):
                th_b = np.clip(ang[offs[k] + b], mesh.lo[k, b], mesh.hi[k, b])
                m = _rot(mesh.axes[k, b], th_b) @ m
            ax = mesh.axes[k, a]
            y = np.cross(ax, m) @ sp
            x = (m - (m @ ax) * ax) @ sp
            if np.hypot(x, y) > 1e-12 * np.linalg.norm(m - (m @ ax) * ax):
                t = np.arctan2(y, x)
                alt = t - np.pi if t > 0 else t + np.pi
                ang[offs[k] + a] = alt if abs(alt) < abs(t) else t
            ang[offs[k] + a] = np.clip(ang[offs[k] + a], mesh.lo[k, a], mesh.hi[k, a])
            sp = _rot(ax, ang[offs[k] + a]).T @ sp
    return ang


def srp_rhs(mesh, mu, mass, p_ref, r_ref, n, bounces=0, track_sun=False, angles0=None, diffuse=0):
    """y' = [v; -mu r/|r|^3 + F/m] with the oracle's ray-traced SRP force at
    the Sun direction -r/|r| and pressure p_ref (r_ref/|r|)^2."""
    state = {"ang": np.zeros(mesh.n_dof) if angles0 is None else np.array(angles0, float)}

    def f(t, y):
        r, v = y[:3], y[3:]
        rn = np.linalg.norm(r)
        s = -r / rn
        if track_sun:
            state["ang"] = sun_tracking(mesh, s, state["ang"])
        P = p_ref * (r_ref / rn) ** 2
        F = eval_srp(mesh, s, n, bounces=bounces, pressure=P, angles=state["ang"], diffuse=diffuse).force
        return np.concatenate([v, -mu * r / rn ** 3 + F / mass])

    return f


def propagate(mesh, y0, t0, h, n_steps, mu, mass, p_ref, r_ref, n, bounces=0, track_sun=False,
              angles0=None):
    """RK4 two-body + ray-traced SRP (oracle forces); returns (n_steps+1, 7)."""
    state = {"ang": np.zeros(mesh.n_dof) if angles0 is None else np.array(angles0, float)}

    def f(t, y):
        r, v = y[:3], y[3:]
        rn = np.linalg.norm(r)
        s = -r / rn
        if track_sun:
            state["ang"] = sun_tracking(mesh, s, state["ang"])
        P = p_ref * (r_ref / rn) ** 2
        F = eval_srp(mesh, s, n, bounces=bounces, pressure=P, angles=state["ang"]).force
        return np.concatenate([v, -mu * r / rn ** 3 + F / mass])

    return rk4(f, y0, t0, h, n_steps)
