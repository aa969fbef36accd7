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
