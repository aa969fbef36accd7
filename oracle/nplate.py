"""FP64 reference for the N-plate model — TEST INFRASTRUCTURE ONLY.

The N-plate model (the analytical SRP model the paper contrasts with ray
tracing, Sec. 1; one of the strategies compared in Sec. 6.1 and 7.1) written
out plainly:

  * plates: every articulated triangle of non-zero area is a plate (area,
    centroid, unit normal from the winding (v1 - v0) x (v2 - v0), the
    triangle's material); plates of panel nodes are lit from either side,
    the others only on their normal's side.  The model is linear in the
    plates, so merging coplanar triangles of one node and material into one
    plate (as a plate list would) changes nothing but rounding.
  * force: per lit plate, s the unit Sun direction, d = -s, n the normal
    turned towards the Sun, c = n . s > 0:
        F = P A c [(1 - rho_s) d - 2 (rho_s c + rho_d / 3) n],
        tau = (centroid - ref) x F;
    no shadowing, no secondary rays.
  * propagation: two-body + N-plate SRP, the attitude fixed (body frame =
    inertial frame), Sun direction -r/|r|, pressure p_ref (r_ref / |r|)^2.
"""
from __future__ import annotations

import numpy as np

from .core import articulate
from .propagate import rk4, rk78

PLATE_DTYPE = np.dtype([("normal", "<f8", 3), ("center", "<f8", 3), ("area", "<f8"), ("rho_s", "<f8"),
                        ("rho_d", "<f8"), ("two_sided", "<i4"), ("reserved", "<i4")])


def plates(mesh, angles=None) -> np.ndarray:
    """One plate per articulated triangle of non-zero area (PLATE_DTYPE)."""
    w = articulate(mesh, angles)                      # (T, 3, 3)
    cr = np.cross(w[:, 1] - w[:, 0], w[:, 2] - w[:, 0])
    ln = np.linalg.norm(cr, axis=1)
    keep = ln > 0
    out = np.zeros(int(keep.sum()), PLATE_DTYPE)
    out["normal"] = cr[keep] / ln[keep, None]
    out["center"] = w[keep].mean(axis=1)
    out["area"] = 0.5 * ln[keep]
    mats = np.asarray(mesh.mats, float)[np.asarray(mesh.tri_mat)[keep]]
    out["rho_s"], out["rho_d"] = mats[:, 0], mats[:, 1]
    out["two_sided"] = np.asarray(mesh.is_panel)[np.asarray(mesh.tri_node)[keep]] != 0
    return out


def force(pl, sun_dir, pressure=1.0, ref=(0.0, 0.0, 0.0)):
    """(force, torque) of the plates for Sun direction sun_dir."""
    s = np.asarray(sun_dir, float)
    s = s / np.linalg.norm(s)
    F, T = np.zeros(3), np.zeros(3)
    for p in pl:
        n = np.array(p["normal"], float)
        c = float(n @ s)
        if c < 0 and p["two_sided"]:
            n, c = -n, -c
        if not c > 0:
            continue
        f = pressure * p["area"] * c * ((1 - p["rho_s"]) * (-s) - 2 * (p["rho_s"] * c + p["rho_d"] / 3) * n)
        F += f
        T += np.cross(np.array(p["center"]) - np.asarray(ref, float), f)
    return F, T


def _rhs(pl, mu, mass, p_ref, r_ref):
    def f(t, y):
        r, v = y[:3], y[3:]
        rn = np.linalg.norm(r)
        F, _ = force(pl, -r / rn, p_ref * (r_ref / rn) ** 2)
        return np.concatenate([v, -mu * r / rn ** 3 + F / mass])
    return f


def propagate(pl, y0, t0, h, n_steps, mu, mass, p_ref, r_ref):
    """RK4 two-body + N-plate SRP; rows (t, r, v)."""
    return rk4(_rhs(pl, mu, mass, p_ref, r_ref), y0, t0, h, n_steps)


def propagate_rk78(pl, y0, t0, t1, h0, mu, mass, p_ref, r_ref, rtol=0.0, atol=None, adaptive=False):
    """RK7(8) two-body + N-plate SRP; (rows (t, r, v) of the accepted steps,
    derivative evaluations)."""
    return rk78(_rhs(pl, mu, mass, p_ref, r_ref), y0, t0, t1, h0, rtol=rtol, atol=atol, adaptive=adaptive)
