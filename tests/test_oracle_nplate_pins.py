"""Pins of the oracle's N-plate model (the analytical model of Sec. 1, one of
the strategies compared in Sec. 6.1 and 7.1).

Pinned by textbook special cases of a plate facing the Sun head-on (a black
plate takes the photons' momentum, a mirror twice that, a Lambertian diffuser
1 + 2/3 of it), by a closed absorbing cube whose lit faces must sum to its
silhouette for any Sun direction (one-sided plates, outward winding), by the
symmetry of a two-sided plate, by splitting a plate (force and torque are
linear in the plates), and by the ray tracer itself where nothing shadows
anything and there is no secondary ray (the box-wing lit face-on)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import nplate as NP

P = 4.56e-6


def _plate(n, c, a, rs, rd, two=0):
    p = np.zeros(1, NP.PLATE_DTYPE)
    p["normal"], p["center"], p["area"], p["rho_s"], p["rho_d"], p["two_sided"] = n, c, a, rs, rd, two
    return p


@pytest.mark.parametrize("rs,rd,mag", [(0.0, 0.0, 1.0), (1.0, 0.0, 2.0), (0.0, 1.0, 1.0 + 2.0 / 3.0)])
def test_head_on_plate(rs, rd, mag):
    s = np.array([0.0, 0.0, 1.0])
    F, T = NP.force(_plate(s, (0, 0, 0), 3.0, rs, rd), s, P)
    np.testing.assert_allclose(F, -mag * P * 3.0 * s, rtol=1e-15, atol=1e-30)
    np.testing.assert_allclose(T, 0.0, atol=1e-30)


def test_one_sided_back_face_and_two_sided_symmetry():
    n = np.array([0.6, 0.0, 0.8])
    for s in (np.array([0.0, 0.3, -1.0]), np.array([-1.0, 0.2, 0.1])):
        F, _ = NP.force(_plate(n, (1, 2, 3), 2.0, 0.3, 0.2), s, P)
        assert np.all(F == 0.0)
        F1, T1 = NP.force(_plate(n, (1, 2, 3), 2.0, 0.3, 0.2, two=1), s, P)
        F2, T2 = NP.force(_plate(n, (1, 2, 3), 2.0, 0.3, 0.2, two=1), -s, P)
        assert np.linalg.norm(F1) > 0
        np.testing.assert_allclose(F2, -F1, rtol=1e-14)
        np.testing.assert_allclose(T2, -T1, rtol=1e-14)


def test_closed_absorbing_cube_gives_its_silhouette():
    """A 1 m cube (outward-wound box of the scene builder), black: F = P A_sil d
    with A_sil = |s_x| + |s_y| + |s_z| for any Sun direction s."""
    m = synth.box_wing(rho_bus=(0.0, 0.0), rho_panel=(0.0, 0.0))
    pl = NP.plates(m)
    bus = pl[np.asarray(pl["two_sided"]) == 0]
    assert len(bus) == 12
    for s in synth.random_dirs(4401, 8):
        F, _ = NP.force(bus, s, P)
        np.testing.assert_allclose(F, -P * np.abs(s).sum() * s, rtol=1e-13, atol=1e-22)


def test_splitting_a_plate_changes_nothing():
    n = np.array([0.0, 0.6, 0.8])
    s = np.array([0.2, 0.5, 0.84])
    whole = _plate(n, (0.5, 1.0, 0.0), 2.0, 0.4, 0.3)
    halves = np.concatenate([_plate(n, (0.0, 1.0, 0.0), 1.0, 0.4, 0.3), _plate(n, (1.0, 1.0, 0.0), 1.0, 0.4, 0.3)])
    ref = np.array([0.3, -0.2, 0.1])
    Fw, Tw = NP.force(whole, s, P, ref)
    Fh, Th = NP.force(halves, s, P, ref)
    np.testing.assert_allclose(Fh, Fw, rtol=1e-14)
    np.testing.assert_allclose(Th, Tw, rtol=1e-14)


def test_equals_the_ray_tracer_without_shadows():
    """Box-wing with the panels flat and the Sun along +z: no face shadows
    another and no ray reflects onto the craft (B = 0), so the ray-traced
    estimator converges to the N-plate force as the grid refines."""
    m = synth.box_wing()
    s = np.array([0.0, 0.0, 1.0])
    F_np, T_np = NP.force(NP.plates(m, np.zeros(2)), s, P, ref=(0.1, 0.2, 0.0))
    errs = []
    for n in (128, 512):
        r = oracle.eval_srp(m, s, n, bounces=0, pressure=P, ref=(0.1, 0.2, 0.0), angles=np.zeros(2))
        errs.append(np.linalg.norm(r.force - F_np) / np.linalg.norm(F_np))
        np.testing.assert_allclose(r.torque, T_np, rtol=0.05, atol=1e-3 * np.linalg.norm(T_np))
    assert errs[1] < 2e-3 and errs[1] <= errs[0], errs


def test_no_plates_is_two_body():
    AU, MU = 1.495978707e11, 1.32712440018e20
    y0 = np.array([AU, 0, 0, 0, np.sqrt(MU / AU), 0])
    a = NP.propagate(np.zeros(0, NP.PLATE_DTYPE), y0, 0.0, 3600.0, 30, MU, 100.0, P, AU)
    from oracle.propagate import rk4
    b = rk4(lambda t, y: np.concatenate([y[3:], -MU * y[:3] / np.linalg.norm(y[:3]) ** 3]), y0, 0.0, 3600.0, 30)
    np.testing.assert_array_equal(a, b)
