"""Pins of the oracle's SPAD table, interpolation and propagation.

The interpolation is pinned by functions it must reproduce exactly (bilinear
in azimuth and elevation), by its behaviour at the azimuth seam and beyond the
sampled elevations; the table by its definition (each node is the oracle's
evaluation at that node's direction, whose axes are fixed by hand); the
propagation by a table filled with the cannonball law F = -k s, whose exact
motion is Kepler's with mu reduced by k P / m, and whose interpolation error
must shrink with the square of the grid spacing."""
import numpy as np
import pytest

import oracle
import synth
from oracle import spad
from oracle.propagate import rk4

DEG = np.pi / 180
AU = 1.495978707e11
MU_SUN = 1.32712440018e20


def test_direction_axes():
    np.testing.assert_allclose(spad.direction(0, 0), [1, 0, 0], atol=1e-16)
    np.testing.assert_allclose(spad.direction(np.pi / 2, 0), [0, 1, 0], atol=1e-16)
    np.testing.assert_allclose(spad.direction(-np.pi / 2, 0), [0, -1, 0], atol=1e-16)
    np.testing.assert_allclose(spad.direction(0.3, np.pi / 2), [0, 0, 1], atol=1e-16)
    np.testing.assert_allclose(spad.direction(np.pi, -np.pi / 4), [-np.sqrt(.5), 0, -np.sqrt(.5)], atol=1e-16)


def _grid(n_az, n_el, az0, el0, daz, de):
    return (n_az, n_el, az0, el0, daz, de)


def test_reproduces_bilinear_functions():
    """A table sampled from f = a + b az + c el + d az el is reproduced
    exactly anywhere inside a non-periodic grid."""
    g = _grid(8, 5, -1.0, -0.5, 0.2, 0.25)
    A = np.array([0.3, -1.2, 0.7, 2.5, -0.4, 1.1])
    Bc = np.array([1.0, 0.5, -2.0, 0.1, 0.0, 3.0])
    Cc = np.array([-0.7, 2.0, 0.3, 1.5, 1.0, -1.0])
    Dc = np.array([0.25, -0.5, 1.0, 0.0, 2.0, 0.7])
    f = lambda az, el: A + Bc * az + Cc * el + Dc * az * el  # noqa: E731
    tab = np.array([[f(g[2] + j * g[4], g[3] + i * g[5]) for j in range(g[0])] for i in range(g[1])])
    rng = np.random.default_rng(7)
    for _ in range(200):
        az = rng.uniform(g[2], g[2] + (g[0] - 1) * g[4])
        el = rng.uniform(g[3], g[3] + (g[1] - 1) * g[5])
        np.testing.assert_allclose(spad.interp(g, tab, 2.5 * spad.direction(az, el)), f(az, el),
                                   rtol=1e-12, atol=1e-12)


def test_nodes_seam_and_held_rows():
    """At a node the table value comes back; across the azimuth seam of a
    periodic grid the last and first columns are blended linearly; beyond the
    sampled elevations the edge row is held."""
    g = _grid(20, 10, -180 * DEG, -90 * DEG, 18 * DEG, 18 * DEG)
    rng = np.random.default_rng(8)
    tab = rng.normal(size=(10, 20, 6))
    for i, j in ((0, 0), (3, 7), (5, 19), (9, 11)):
        s = spad.direction(g[2] + j * g[4], g[3] + i * g[5])
        np.testing.assert_allclose(spad.interp(g, tab, s), tab[i, j], rtol=1e-12, atol=1e-12)
    # between azimuth 162 (column 19) and 180 = -180 (column 0), on the 0 deg row (5)
    for t in (0.25, 0.5, 0.9):
        s = spad.direction((162 + 18 * t) * DEG, 0.0)
        np.testing.assert_allclose(spad.interp(g, tab, s), (1 - t) * tab[5, 19] + t * tab[5, 0], rtol=1e-11, atol=1e-12)
    # above the last row (72 deg) and below the first (-90 deg is the pole: the row itself)
    s = spad.direction(-171 * DEG, 81 * DEG)
    np.testing.assert_allclose(spad.interp(g, tab, s), 0.5 * (tab[9, 0] + tab[9, 1]), rtol=1e-11, atol=1e-12)
    gs = _grid(20, 10, -175 * DEG, -85 * DEG, 18 * DEG, 18 * DEG)
    s = spad.direction(-175 * DEG, -88 * DEG)
    np.testing.assert_allclose(spad.interp(gs, tab, s), tab[0, 0], rtol=1e-11, atol=1e-12)


def test_table_nodes_are_evaluations():
    """Each node of the table is the oracle's evaluation at that node's
    direction (bitwise), for the box-wing at a hinge setting."""
    mesh = synth.box_wing()
    g = _grid(5, 3, -180 * DEG, -36 * DEG, 72 * DEG, 36 * DEG)
    ang = np.array([0.4, -0.3])
    tab = spad.table(mesh, g, 24, bounces=1, pressure=2.0, angles=ang, ref=(0.1, 0, 0))
    for i in range(3):
        for j in range(5):
            r = oracle.eval_srp(mesh, spad.direction(g[2] + j * g[4], g[3] + i * g[5]), 24, bounces=1,
                                pressure=2.0, angles=ang, ref=(0.1, 0, 0))
            assert tab[i, j, :3].tobytes() == r.force.tobytes() and tab[i, j, 3:].tobytes() == r.torque.tobytes()


def _cannonball_table(g, k):
    return np.array([[np.concatenate([-k * spad.direction(g[2] + j * g[4], g[3] + i * g[5]), np.zeros(3)])
                      for j in range(g[0])] for i in range(g[1])])


@pytest.mark.parametrize("shift", [0.0, 5.0 / 18.0])
def test_spad_propagation_converges_with_the_grid(shift):
    """Cannonball table F = -k s at pressure p_table: the exact motion is
    Kepler's with mu' = mu - k p(r) r^2 / (m p_table) (p ~ 1/r^2).  SPAD
    propagation over one circular orbit (a = 0.388 AU, Sec. 6.1 table of
    orbits) has a position error that shrinks about 16-fold when the spacing
    drops from 18 to 4.5 deg (bilinear interpolation error ~ spacing^2); the
    shifted grids start `shift` spacings past -180 / -90 deg (5 deg at 18)."""
    k, mass, p_ref, r_ref = 3.0e3, 500.0, 4.56e-6, AU
    a = 0.388 * AU
    v = np.sqrt(MU_SUN / a)
    y0 = np.array([a, 0, 0, 0, v, 0])
    T = 2 * np.pi * np.sqrt(a ** 3 / MU_SUN)
    n_steps = 400
    h = T / n_steps
    mu_eff = MU_SUN - k * p_ref * r_ref ** 2 / mass
    ref = rk4(lambda t, y: np.concatenate([y[3:], -mu_eff * y[:3] / np.linalg.norm(y[:3]) ** 3]), y0, 0.0, h, n_steps)
    errs = []
    for d in (18.0, 4.5):
        n_az, n_el = int(round(360 / d)), int(round(180 / d))
        g = _grid(n_az, n_el, (-180 + shift * d) * DEG, (-90 + shift * d) * DEG, d * DEG, d * DEG)
        tab = _cannonball_table(g, k)
        tr = spad.propagate(g, tab, 1.0, y0, 0.0, h, n_steps, MU_SUN, mass, p_ref, r_ref)
        errs.append(np.linalg.norm(tr[-1, 1:4] - ref[-1, 1:4]))
    # the SRP displacement itself: Kepler with the full mu
    kep = rk4(lambda t, y: np.concatenate([y[3:], -MU_SUN * y[:3] / np.linalg.norm(y[:3]) ** 3]), y0, 0.0, h, n_steps)
    srp_shift = np.linalg.norm(kep[-1, 1:4] - ref[-1, 1:4])
    assert errs[0] < 0.1 * srp_shift, (errs, srp_shift)
    assert 12 < errs[0] / errs[1] < 20, errs


def test_zero_table_is_two_body():
    g = _grid(20, 10, -180 * DEG, -90 * DEG, 18 * DEG, 18 * DEG)
    a = 0.557 * AU
    y0 = np.array([a * (1 - 0.682), 0, 0, 0, np.sqrt(MU_SUN * (1 + 0.682) / (a * (1 - 0.682))), 0])
    tr = spad.propagate(g, np.zeros((10, 20, 6)), 1.0, y0, 0.0, 3600.0, 50, MU_SUN, 100.0, 4.56e-6, AU)
    kep = rk4(lambda t, y: np.concatenate([y[3:], -MU_SUN * y[:3] / np.linalg.norm(y[:3]) ** 3]), y0, 0.0, 3600.0, 50)
    np.testing.assert_array_equal(tr, kep)
