"""FP64 reference for SPAD tables — TEST INFRASTRUCTURE ONLY.

A SPAD table (Sec. 2 and Sec. 4.2 of the paper: SRP precomputed offline over
spacecraft attitudes and interpolated during propagation; Sec. 6.1: grids of
20 azimuth x 10 elevation values from -180 / -90 deg, and a copy shifted by
5 deg) written out plainly:

  * grid: az_j = az0 + j daz (j < n_az), el_i = el0 + i del (i < n_el); node
    (i, j) holds the SRP force and torque for the Sun direction, in the body
    frame, s(az, el) = (cos el cos az, cos el sin az, sin el), at fixed hinge
    angles and a given pressure.  The paper's 20 x 10 grids and the remark
    that only the unshifted one has samples at 0 deg elevation fit a spacing
    of 18 deg on both axes (azimuth -180..162, elevation -90..72).
  * interpolation: the direction's azimuth atan2(s_y, s_x) and elevation
    atan2(s_z, hypot(s_x, s_y)); bilinear in (az, el) between the four
    surrounding nodes; azimuth wraps around when n_az daz = 360 deg (else it
    is held at the first / last column), elevation beyond the first / last
    row is held at that row.
  * propagation: the force scales with the pressure, p(r) / p_table.
"""
from __future__ import annotations

import numpy as np

from .core import eval_srp
from .propagate import rk4

TWO_PI = 2.0 * np.pi


def direction(az, el):
    """Body-frame Sun direction of azimuth az and elevation el (radians)."""
    return np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])


def table(mesh, grid, n, bounces=0, pressure=1.0, ref=(0, 0, 0), angles=None, diffuse=0):
    """(n_el, n_az, 6) force and torque at every grid direction (oracle rays)."""
    n_az, n_el, az0, el0, daz, de = grid
    out = np.zeros((n_el, n_az, 6))
    for i in range(n_el):
        for j in range(n_az):
            r = eval_srp(mesh, direction(az0 + j * daz, el0 + i * de), n, bounces=bounces,
                         pressure=pressure, ref=ref, angles=angles, diffuse=diffuse)
            out[i, j, :3], out[i, j, 3:] = r.force, r.torque
    return out


def periodic(grid):
    n_az, _, _, _, daz, _ = grid
    return abs(n_az * daz - TWO_PI) <= 1e-9


def interp(grid, tab, s):
    """Bilinear interpolation of the table at Sun direction s (6 values)."""
    n_az, n_el, az0, el0, daz, de = grid
    s = np.asarray(s, float)
    az = np.arctan2(s[1], s[0])
    el = np.arctan2(s[2], np.hypot(s[0], s[1]))
    u = (az - az0) / daz
    if periodic(grid):
        u = u % n_az                       # in [0, n_az)
        j0 = int(np.floor(u))
        fu = u - j0
        j0 %= n_az
        j1 = (j0 + 1) % n_az
    else:
        u = min(max(u, 0.0), n_az - 1.0)
        j0 = min(int(np.floor(u)), max(n_az - 2, 0))
        fu = u - j0
        j1 = min(j0 + 1, n_az - 1)
    v = min(max((el - el0) / de, 0.0), n_el - 1.0)
    i0 = min(int(np.floor(v)), max(n_el - 2, 0))
    fv = v - i0
    i1 = min(i0 + 1, n_el - 1)
    return ((1 - fu) * (1 - fv) * tab[i0, j0] + fu * (1 - fv) * tab[i0, j1]
            + (1 - fu) * fv * tab[i1, j0] + fu * fv * tab[i1, j1])


def propagate(grid, tab, p_table, y0, t0, h, n_steps, mu, mass, p_ref, r_ref):
    """RK4 two-body + SRP with the force interpolated from the table at the
    stage's Sun direction -r/|r| and scaled to the stage's pressure."""

    def f(t, y):
        r, v = y[:3], y[3:]
        rn = np.linalg.norm(r)
        P = p_ref * (r_ref / rn) ** 2
        F = interp(grid, tab, -r / rn)[:3] * (P / p_table)
        return np.concatenate([v, -mu * r / rn ** 3 + F / mass])

    return rk4(f, y0, t0, h, n_steps)
