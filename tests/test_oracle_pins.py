"""Pins of the FP64 oracle against closed forms, invariants and brute force.

The paper prints no force value for a worked example, so every pin below is
fixed by geometry and mechanics, derived by hand in each docstring.  They
are chosen so that a plausible mistake in the oracle (a dropped term of the
law, a wrong sign or orientation of the normal, a transposed rotation, a
wrong window or pixel area, a broken tie rule, a secondary ray that keeps or
loses weight wrongly, an acceleration structure that drops a triangle)
fails at least one of them.

Notation: d = photon direction (= -sun_dir), n = unit normal facing the
incoming ray, c = -n.d, P = pressure, A_proj = projected area.
Flat-plate law per unit projected area: (1-rs) d - 2 (rs c + rd/3) n.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _basis(d):
    """Image-plane axes for photon direction d (the reading the oracle uses:
    helper e_z unless |d_z| >= 0.9, then e_x; u = h x d normalised, v = d x u)."""
    h = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    u = np.cross(h, d)
    u /= np.linalg.norm(u)
    return u, np.cross(d, u)


def _aligned_plate(sun, a, b, tilt, rho):
    """Plate whose projection fills its window exactly: one edge along u
    (length a), the other (length b) in the (v, d) plane at angle `tilt` from v.
    Its unit normal is u x (cos t v + sin t d), |n.d| = cos(tilt)."""
    d = -np.asarray(sun, float) / np.linalg.norm(sun)
    u, v = _basis(d)
    eu = a * u
    ev = b * (np.cos(tilt) * v + np.sin(tilt) * d)
    return synth.plate(origin=0.3 * u - 0.7 * v + 0.2 * d, eu=eu, ev=ev, rho=rho), d, u, v


@pytest.mark.parametrize("seed", [11, 12, 13])
@pytest.mark.parametrize("n", [16, 33])
def test_flat_plate_closed_form(seed, n):
    """All N^2 rays hit the plate, so F = P A cos(t) [(1-rs) d - 2 (rs cos t + rd/3) n]
    with A = a b and n facing the ray.  Holds exactly (to rounding) for any N."""
    rng = np.random.default_rng(seed)
    sun = synth.random_dirs(seed)[0]
    a, b, tilt = rng.uniform(0.5, 3), rng.uniform(0.5, 3), rng.uniform(-1.2, 1.2)
    rs, rd = rng.uniform(0, 0.5), rng.uniform(0, 0.5)
    P = rng.uniform(0.5, 5)
    sc, d, u, v = _aligned_plate(sun, a, b, tilt, (rs, rd))
    nrm = np.cross(u, np.cos(tilt) * v + np.sin(tilt) * d)
    if nrm @ d > 0:
        nrm = -nrm
    cth = -nrm @ d
    assert abs(cth - np.cos(tilt)) < 1e-12
    F = P * a * b * cth * ((1 - rs) * d - 2 * (rs * cth + rd / 3) * nrm)
    r = oracle.eval_srp(sc, sun, n, bounces=2, pressure=P)
    assert r.n_hits == n * n
    assert r.n_secondary_hits == 0          # a single plane cannot be hit twice
    np.testing.assert_allclose(r.force, F, rtol=1e-12, atol=1e-12 * np.abs(F).max())
    # projected area is carried by the pixels: N^2 A_pix = a b cos(t)
    assert abs(n * n * r.grid["a_pix"] - a * b * cth) < 1e-12 * a * b


def test_flat_plate_torque_closed_form():
    """Torque about ref of a uniformly hit plate: (x_c - ref) x F where x_c is
    the centroid of the hit points, i.e. the plate's centre (pixel centres are
    symmetric about it)."""
    sun = synth.random_dirs(21)[0]
    sc, d, u, v = _aligned_plate(sun, 2.0, 1.5, 0.4, (0.3, 0.2))
    ref = np.array([0.5, -1.0, 2.0])
    r = oracle.eval_srp(sc, sun, 32, bounces=0, ref=ref)
    centre = sc.verts.mean(0)
    np.testing.assert_allclose(r.torque, np.cross(centre - ref, r.force), rtol=1e-11,
                               atol=1e-11 * np.linalg.norm(r.torque))


@pytest.mark.parametrize("rho", [(0.0, 0.0), (0.2, 0.4), (0.7, 0.1)])
def test_cube_face_on(rho):
    """Sun along +z onto a cube: only the +z face is hit (side faces are edge-on
    and rejected as grazing), c = 1, n = -d:  F = P A (1 + rs + 2 rd/3) d."""
    rs, rd = rho
    sc = synth.cube(half=0.75, rho=rho)
    r = oracle.eval_srp(sc, (0, 0, 1), 24, bounces=1, pressure=2.0)
    d = np.array([0.0, 0.0, -1.0])
    F = 2.0 * 1.5 * 1.5 * (1 + rs + 2 * rd / 3) * d
    np.testing.assert_allclose(r.force, F, rtol=1e-12, atol=1e-13)
    assert r.n_hits == 24 * 24


@pytest.mark.parametrize("rho", [(1.0, 0.0), (0.5, 0.3), (0.2, 0.0), (0.0, 0.6)])
@pytest.mark.parametrize("bounces", [0, 1, 2])
def test_dihedral_retroreflector(rho, bounces):
    """Two L x H faces at 90 deg, d = -(0,1,1)/sqrt2 at 45 deg to both; the
    projections of the faces tile the window (area sqrt2 L H), half the rays
    hit each face first with c = 1/sqrt2, reflect onto the other face (again
    c = 1/sqrt2) and leave along -d.  Summing the two hits of both halves with
    y + z = -sqrt2 d and d' + d'' = 0:
        B = 0:  F = sqrt2 L H P [1 + (sqrt2/3) rd] d
        B >= 1: F = sqrt2 L H P [1 + rs^2 + (sqrt2/3)(1 + rs) rd] d
    With rs = 1, rd = 0, B >= 1 this is the perfect retroreflector 2 P A d."""
    rs, rd = rho
    L, H, P = 1.3, 0.7, 1.7
    sc = synth.dihedral(L, H, rho)
    sun = np.array([0.0, 1.0, 1.0]) / np.sqrt(2)
    d = -sun
    r = oracle.eval_srp(sc, sun, 40, bounces=bounces, pressure=P)
    A = np.sqrt(2) * L * H
    if bounces == 0:
        k = 1 + np.sqrt(2) / 3 * rd
    else:
        k = 1 + rs ** 2 + np.sqrt(2) / 3 * (1 + rs) * rd
    np.testing.assert_allclose(r.force, A * P * k * d, rtol=1e-12, atol=1e-12)
    if bounces and rs > 0:
        assert r.n_secondary_hits == 40 * 40
    else:
        assert r.n_secondary_hits == 0


def test_black_body_counts_hits():
    """rs = rd = 0: every hit transfers exactly its momentum, dF = P A_pix d, so
    F = P A_pix N_hit d (N_hit an integer) and no secondary ray is spawned."""
    sc = synth.procedural_sized(7, 3000)
    sc = sc.with_mats(np.zeros_like(sc.mats))
    sun = synth.random_dirs(31)[0]
    r = oracle.eval_srp(sc, sun, 96, bounces=2, pressure=3.0, angles=np.full(sc.n_dof, 0.3))
    d = -sun / np.linalg.norm(sun)
    np.testing.assert_allclose(r.force, 3.0 * r.grid["a_pix"] * r.n_hits * d, rtol=1e-12)
    assert r.n_secondary == 0 and 0 < r.n_hits < 96 * 96


def test_occluded_facet_changes_nothing():
    """A facet inside a closed cube (inside the footprint, so the window is
    unchanged) is never the first hit: F, tau and the primary ids are
    bitwise unchanged."""
    base = synth.cube(half=1.0, rho=(0.4, 0.3))
    hidden = np.array([[-0.5, -0.5, 0.0], [0.5, -0.4, 0.2], [0.0, 0.6, -0.3]])
    sc = synth.merge_static(base, np.concatenate([base.verts[base.tris], hidden[None]]),
                            tri_mat=np.zeros(13, np.int32))
    for seed in (41, 42, 43):
        sun = synth.random_dirs(seed)[0]
        for bvh in (False, True):
            a = oracle.eval_srp(base, sun, 48, bounces=2, use_bvh=bvh, record=True)
            b = oracle.eval_srp(sc, sun, 48, bounces=2, use_bvh=bvh, record=True)
            assert np.array_equal(a.force, b.force) and np.array_equal(a.torque, b.torque)
            assert np.array_equal(a.ids, b.ids)


def test_zero_area_triangle_never_hit():
    """A zero-area triangle (two coincident corners) in front of a plate is
    never hit: the result equals the plate alone, bitwise."""
    sun = np.array([0.0, 0.0, 1.0])
    base = synth.plate((-1, -1, 0), (2, 0, 0), (0, 2, 0), rho=(0.3, 0.3))
    degen = np.array([[[-0.5, 0.0, 0.5], [0.5, 0.0, 0.5], [0.5, 0.0, 0.5]]])
    sc = synth.merge_static(base, np.concatenate([base.verts[base.tris], degen]),
                            tri_mat=np.zeros(3, np.int32))
    a = oracle.eval_srp(base, sun, 50, bounces=1)
    b = oracle.eval_srp(sc, sun, 50, bounces=1)
    assert np.array_equal(a.force, b.force) and a.n_hits == b.n_hits == 2500


@pytest.mark.parametrize("subdiv,n,tol", [(3, 256, 2e-2), (5, 1024, 1.5e-3)])
def test_cannonball_limit(subdiv, n, tol):
    """A sphere of radius R: integrating the law over the lit hemisphere,
    int c dA = pi R^2, int c^2 (n.d) dA = -2 pi R^2/3, int c^3 dA = pi R^2/2, so
    F = P pi R^2 [(1-rs) + rs + 4 rd/9] d = P pi R^2 (1 + 4 rd/9) d
    (specular reflection returns exactly the absorbed momentum).  The faceted,
    pixelated estimate converges to it; B = 0 (convex: no secondary hits)."""
    R, rs, rd = 1.3, 0.35, 0.45
    sc = synth.icosphere(R, subdiv, rho=(rs, rd))
    sun = synth.random_dirs(51)[0]
    r = oracle.eval_srp(sc, sun, n, bounces=0)
    d = -sun / np.linalg.norm(sun)
    F = np.pi * R * R * (1 + 4 * rd / 9) * d
    assert np.linalg.norm(r.force - F) / np.linalg.norm(F) < tol


def test_convex_cube_matches_n_plate():
    """For a convex body and B = 0 every lit face is fully visible, so the ray
    estimate converges (as 1/N from the pixelated face outlines) to the
    N-plate sum over lit faces of P A_f c_f [(1-rs) d - 2 (rs c_f + rd/3) n_f]."""
    half, rs, rd = 0.6, 0.25, 0.35
    sc = synth.cube(half, rho=(rs, rd))
    sun = synth.random_dirs(61)[0]
    d = -sun / np.linalg.norm(sun)
    F = np.zeros(3)
    for ax in range(3):
        for sgn in (-1, 1):
            n_out = np.zeros(3)
            n_out[ax] = sgn
            c = -(n_out @ d)
            if c > 0:
                F += (2 * half) ** 2 * c * ((1 - rs) * d - 2 * (rs * c + rd / 3) * n_out)
    errs = []
    for n in (128, 512):
        r = oracle.eval_srp(sc, sun, n, bounces=0)
        errs.append(np.linalg.norm(r.force - F) / np.linalg.norm(F))
    assert errs[1] < 6e-3 and errs[1] < errs[0]


def test_linearity_in_pressure_and_coefficients():
    """F and tau scale with P (exactly, by a power of two); with B = 0 the
    force is affine in (rs, rd) at fixed geometry:
    F(rs,rd) - F(0,0) = rs (F(1,0) - F(0,0)) + rd (F(0,1) - F(0,0))."""
    sc = synth.procedural_sized(8, 2500)
    sun = synth.random_dirs(71)[0]
    ang = np.linspace(-0.4, 0.6, sc.n_dof)
    a = oracle.eval_srp(sc, sun, 64, bounces=2, pressure=1.0, angles=ang)
    b = oracle.eval_srp(sc, sun, 64, bounces=2, pressure=4.0, angles=ang)
    assert np.array_equal(4 * a.force, b.force) and np.array_equal(4 * a.torque, b.torque)

    def F(rs, rd):
        m = np.tile([rs, rd], (sc.n_mats, 1))
        return oracle.eval_srp(sc.with_mats(m), sun, 64, bounces=0, angles=ang).force

    f00, f10, f01, f = F(0, 0), F(1, 0), F(0, 1), F(0.3, 0.45)
    np.testing.assert_allclose(f - f00, 0.3 * (f10 - f00) + 0.45 * (f01 - f00), rtol=1e-11,
                               atol=1e-12 * np.abs(f).max())


@pytest.mark.parametrize("maker,seed,bounces", [
    (lambda: synth.box_wing(), 81, 2),
    (lambda: synth.procedural_sized(9, 1500), 82, 2),
    (lambda: synth.icosphere(1.0, 2), 83, 1),
    (lambda: synth.dihedral(1.0, 2.0, (0.6, 0.2)), 84, 2),
])
def test_bvh_matches_brute_force(maker, seed, bounces):
    """The oracle's acceleration structure returns exactly what the plain loop
    over all triangles returns: identical ids of every generation, identical t
    and bitwise-identical sums."""
    sc = maker()
    ang = np.linspace(-0.5, 0.5, sc.n_dof) if sc.n_dof else None
    for k in range(3):
        sun = synth.random_dirs(seed * 10 + k)[0]
        a = oracle.eval_srp(sc, sun, 40, bounces=bounces, angles=ang, use_bvh=False, record=True)
        b = oracle.eval_srp(sc, sun, 40, bounces=bounces, angles=ang, use_bvh=True, record=True)
        assert np.array_equal(a.ids, b.ids)
        assert np.array_equal(a.ts, b.ts)
        assert np.array_equal(a.force, b.force) and np.array_equal(a.torque, b.torque)


def _Ry(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _Rx(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def test_articulation_by_hand():
    """Node transforms against hand-written rotations: a box-wing panel turns
    about y through (0, 1.5, 0); a procedural wing's second segment turns by
    the root hinge (about y through (0,1.5,0)) composed with its fold (about x
    through (0,3.5,0)).  Points on a hinge line stay put; transforms are rigid;
    angles outside the interval are clamped."""
    bw = synth.box_wing()
    X = oracle.node_transforms(bw, [0.7, -0.2])
    p = np.array([0.3, 4.0, 0.0])
    piv = np.array([0, 1.5, 0])
    np.testing.assert_allclose(X[1, :, :3] @ p + X[1, :, 3], _Ry(0.7) @ (p - piv) + piv, atol=1e-14)
    piv2 = np.array([0, -1.5, 0])
    np.testing.assert_allclose(X[2, :, :3] @ p + X[2, :, 3], _Ry(-0.2) @ (p - piv2) + piv2,
                               atol=1e-14)
    for k in range(3):
        np.testing.assert_allclose(X[k, :, :3].T @ X[k, :, :3], np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(X[k, :, :3]) - 1) < 1e-14
    # clamping (Sec. 4.4.2 step 4): |angle| beyond pi/2 behaves as +-pi/2
    np.testing.assert_allclose(oracle.node_transforms(bw, [5.0, -7.0]),
                               oracle.node_transforms(bw, [np.pi / 2, -np.pi / 2]), atol=0)

    sc = synth.procedural_spacecraft(seed=2, dish_rings=4, dish_sectors=4, seg_nx=2, seg_ny=2)
    ang = np.zeros(sc.n_dof)
    ang[0], ang[1] = 0.6, -0.9            # +y wing: root hinge, first fold
    X = oracle.node_transforms(sc, ang)
    q = np.array([0.4, 4.2, 0.0])         # a point of segment 2 (y in [3.5, 5.5])
    pa, pb = np.array([0, 1.5, 0]), np.array([0, 3.5, 0])
    expect = _Ry(0.6) @ ((_Rx(-0.9) @ (q - pb) + pb) - pa) + pa
    np.testing.assert_allclose(X[2, :, :3] @ q + X[2, :, 3], expect, atol=1e-14)
    # the fold line of segment 2 rotates with the root hinge only
    np.testing.assert_allclose(X[2, :, :3] @ pb + X[2, :, 3], _Ry(0.6) @ (pb - pa) + pa, atol=1e-14)


def test_hinged_plate_follows_flat_plate_law():
    """A panel turned by t about y (the u axis when the sun is on +z, which
    makes its projection fill the window) is a flat plate with c = cos t and
    n = (sin t, 0, cos t) facing the sun."""
    rs, rd = 0.3, 0.25
    sc = synth.hinged_plate(width=2.0, length=3.0, rho=(rs, rd))
    d = np.array([0.0, 0.0, -1.0])
    for t in (-1.1, -0.3, 0.0, 0.5, 1.2):
        r = oracle.eval_srp(sc, (0, 0, 1), 20, bounces=0, angles=[t])
        n = np.array([np.sin(t), 0.0, np.cos(t)])
        c = np.cos(t)
        F = 6.0 * c * ((1 - rs) * d - 2 * (rs * c + rd / 3) * n)
        np.testing.assert_allclose(r.force, F, rtol=1e-12, atol=1e-13)


def test_frozen_shade_reproduces_eval():
    """Re-shading the recorded chains at the recording state gives back the
    traced force (the plane intersection and the triangle test agree on t)."""
    sc = synth.procedural_sized(10, 4000)
    ang = np.linspace(-0.8, 0.8, sc.n_dof)
    sun = synth.random_dirs(91)[0]
    r = oracle.eval_srp(sc, sun, 64, bounces=2, angles=ang, record=True, pressure=2.5)
    s = oracle.shade_frozen(sc, sun, 64, 2, r.grid, r.ids, pressure=2.5, angles=ang)
    np.testing.assert_allclose(s.force, r.force, rtol=1e-11)
    np.testing.assert_allclose(s.torque, r.torque, rtol=1e-10)
    assert s.n_hits == r.n_hits and s.n_secondary_hits == r.n_secondary_hits


def _hinged_plate_force_and_gradient(rs, rd, P, t, A):
    """Flat-plate law of the hinged plate lit along d = -z, written out by
    hand: n(t) = R_y(t) z faces the Sun, c = cos t, so
        F(t)  = P A c [(1-rs) d - 2 (rs c + rd/3) n],
        dF/dt = P A [c' ((1-rs) d - 2 (rs c + rd/3) n) - 2 c (rs c' n + (rs c + rd/3) n')],
    with c' = -sin t and n' = y x n = (cos t, 0, -sin t)."""
    d = np.array([0.0, 0.0, -1.0])
    n = np.array([np.sin(t), 0.0, np.cos(t)])
    c, cp = np.cos(t), -np.sin(t)
    npr = np.array([np.cos(t), 0.0, -np.sin(t)])
    law = (1 - rs) * d - 2 * (rs * c + rd / 3) * n
    F = P * A * c * law
    dF = P * A * (cp * law - 2 * c * (rs * cp * n + (rs * c + rd / 3) * npr))
    return F, dF, d, n, c


def test_flat_plate_gradients_closed_form():
    """Fixed visibility for the hinged plate (every pixel hits it): each ray
    keeps its share of the plate's surface, so the frozen variation is the
    flat-plate law's own, F(t) = P A cos t [...].  The coefficient terms at
    fixed t are dF/drs = P A c (-d - 2 c n) and dF/drd = -(2/3) P A c n; the
    hinge term is the derivative of F(t) including its cos t prefactor
    (_hinged_plate_force_and_gradient).  The same closed form is the central
    difference of the full evaluation re-traced at t +- h (window and pixel
    area re-fitted), which ties the convention to the true force."""
    rs, rd, P = 0.35, 0.2, 1.9
    sc = synth.hinged_plate(2.0, 3.0, rho=(rs, rd))
    sun = np.array([0.0, 0.0, 1.0])
    for t in (0.45, -0.8, 1.1):
        F, dF, d, n, c = _hinged_plate_force_and_gradient(rs, rd, P, t, 6.0)
        r = oracle.eval_srp(sc, sun, 16, bounces=1, pressure=P, angles=[t], record=True)
        np.testing.assert_allclose(r.force, F, rtol=1e-12, atol=1e-13)
        g = oracle.fd_gradients(sc, sun, 16, 1, r.grid, r.ids, pressure=P, angles=[t])
        np.testing.assert_allclose(g["rho_s"][0], P * 6.0 * c * (-d - 2 * c * n), rtol=1e-8, atol=1e-9)
        np.testing.assert_allclose(g["rho_d"][0], -2 / 3 * P * 6.0 * c * n, rtol=1e-8, atol=1e-9)
        np.testing.assert_allclose(g["theta"][0], dF, rtol=1e-7, atol=1e-8 * np.abs(dF).max())
        h = 1e-5
        fp = oracle.eval_srp(sc, sun, 16, bounces=1, pressure=P, angles=[t + h]).force
        fm = oracle.eval_srp(sc, sun, 16, bounces=1, pressure=P, angles=[t - h]).force
        np.testing.assert_allclose((fp - fm) / (2 * h), dF, rtol=1e-7, atol=1e-8 * np.abs(dF).max())


def test_frozen_share_is_one_at_the_recorded_angles():
    """With the recorded angles as reference the surface-share factor is
    exactly 1, so the re-shade gives the plain re-shade's force and torque
    bitwise.  A lone plate recorded head-on (t = 0) and turned by dt keeps
    every ray on it, each with its share of the surface, so the frozen force
    is the flat-plate law at dt, cos(dt) prefactor included."""
    sc = synth.procedural_sized(13, 3000)
    ang = np.linspace(-0.7, 0.6, sc.n_dof)
    sun = synth.random_dirs(93)[0]
    r = oracle.eval_srp(sc, sun, 48, bounces=2, angles=ang, record=True)
    a = oracle.shade_frozen(sc, sun, 48, 2, r.grid, r.ids, angles=ang)
    b = oracle.shade_frozen(sc, sun, 48, 2, r.grid, r.ids, angles=ang, angles_ref=ang)
    assert np.array_equal(a.force, b.force) and np.array_equal(a.torque, b.torque)
    # a lone plate lit head-on (t = 0), turned by dt under frozen visibility:
    # F(dt) = P A cos(dt) [(1-rs) d - 2 (rs cos dt + rd/3) n(dt)] exactly
    rs, rd = 0.3, 0.25
    hp = synth.hinged_plate(2.0, 3.0, rho=(rs, rd))
    rr = oracle.eval_srp(hp, (0, 0, 1), 12, bounces=0, angles=[0.0], record=True)
    for dt in (0.2, -0.5):
        F, _, _, _, _ = _hinged_plate_force_and_gradient(rs, rd, 1.0, dt, 6.0)
        got = oracle.shade_frozen(hp, (0, 0, 1), 12, 0, rr.grid, rr.ids, angles=[dt], angles_ref=[0.0])
        np.testing.assert_allclose(got.force, F, rtol=1e-12, atol=1e-13)


def test_frozen_share_holds_the_face_met():
    """Fixed visibility holds the face each recorded ray met.  A plate hinged
    about y, lit from s = (sin a, 0, cos a) (a = -0.3), has c(t) = n(t).s =
    cos(t - a); recorded at t = 1.2 (c = 0.071) and re-shaded at t = 1.35 it
    has turned past edge-on (c = -0.079).  With the recorded face held, the
    frozen force is the flat-plate law continued through edge-on,
    P A c(t) [(1-rs) d - 2 (rs c(t) + rd/3) n(t)] with n(t) = R_y(t) z and
    c(t) < 0, and the central difference across edge-on is its derivative
    (re-orienting the normal toward the ray would flip the rd term and put a
    kink at edge-on)."""
    rs, rd, P, a = 0.3, 0.25, 1.4, -0.3
    sc = synth.hinged_plate(2.0, 3.0, rho=(rs, rd))
    sun = np.array([np.sin(a), 0.0, np.cos(a)])
    d = -sun

    def law(t):
        n = np.array([np.sin(t), 0.0, np.cos(t)])
        c = np.cos(t - a)
        return P * 6.0 * c * ((1 - rs) * d - 2 * (rs * c + rd / 3) * n)

    r = oracle.eval_srp(sc, sun, 16, bounces=0, pressure=P, angles=[1.2], record=True)
    assert r.n_hits == 256
    np.testing.assert_allclose(r.force, law(1.2), rtol=1e-11, atol=1e-13)
    for t in (1.35, 1.27):
        got = oracle.shade_frozen(sc, sun, 16, 0, r.grid, r.ids, pressure=P, angles=[t], angles_ref=[1.2])
        np.testing.assert_allclose(got.force, law(t), rtol=1e-11, atol=1e-13)
    h = 1e-4
    t0 = np.pi / 2 + a            # exactly edge-on
    fd = (oracle.shade_frozen(sc, sun, 16, 0, r.grid, r.ids, pressure=P, angles=[t0 + h], angles_ref=[1.2]).force -
          oracle.shade_frozen(sc, sun, 16, 0, r.grid, r.ids, pressure=P, angles=[t0 - h], angles_ref=[1.2]).force)
    np.testing.assert_allclose(fd / (2 * h), (law(t0 + 1e-6) - law(t0 - 1e-6)) / 2e-6, rtol=1e-6, atol=1e-9)


def test_paper_material_tables():
    """The printed optical coefficients satisfy p_s + p_d + p_a = 1 for every
    part; the oracle accepts them and rejects a row with rs + rd > 1."""
    tab = json.load(open(os.path.join(GOLD, "paper_tables.json")))
    rows = [v for sc in tab["materials"].values() for v in sc.values()]
    for rs, rd, ra in rows:
        assert abs(rs + rd + ra - 1) < 1e-12
    bw = synth.box_wing(rho_bus=tuple(tab["materials"]["BoxWing"]["bus"][:2]),
                        rho_panel=tuple(tab["materials"]["BoxWing"]["solar array"][:2]))
    r = oracle.eval_srp(bw, (0.3, 0.2, 0.9), 32, bounces=2)
    assert np.isfinite(r.force).all() and r.n_hits > 0
    with pytest.raises(ValueError):
        oracle.eval_srp(bw.with_mats([[0.6, 0.5], [0.1, 0.1]]), (0, 0, 1), 8)


def test_empty_window_and_bad_inputs():
    """An edge-on single plate has a zero-area window: F = tau = 0 and no hit.
    A zero sun direction is rejected."""
    sc = synth.plate((0, 0, 0), (1, 0, 0), (0, 1, 0))
    r = oracle.eval_srp(sc, (1, 0, 0), 16, bounces=1)
    assert r.n_hits == 0 and not r.force.any() and not r.torque.any()
    with pytest.raises(ValueError):
        oracle.eval_srp(sc, (0, 0, 0), 16)


def test_pixel_subset_matches_full_grid():
    """Tracing a listed subset of pixels gives, per pixel, the ids of the full
    run (used for sampled parity at full sizes)."""
    sc = synth.procedural_sized(12, 2000)
    sun = synth.random_dirs(95)[0]
    full = oracle.eval_srp(sc, sun, 48, bounces=2, record=True)
    pix = np.random.default_rng(0).choice(48 * 48, 300, replace=False)
    sub = oracle.eval_srp(sc, sun, 48, bounces=2, pixels=pix, record=True)
    assert np.array_equal(sub.ids, full.ids[pix]) and np.array_equal(sub.ts, full.ts[pix])


def test_exact_tie_goes_to_lowest_index():
    """The same triangle listed twice with different materials: both copies are
    hit at exactly the same t by every ray, and the copy with the lower index
    takes the hit, so the force is that of its material alone."""
    base = synth.plate((-1, -1, 0), (2, 0, 0), (0, 2, 0), rho=(0.0, 0.0))
    tv = base.verts[base.tris]
    mats = np.array([[0.5, 0.1], [0.0, 0.0]])
    both = synth.merge_static(base, np.concatenate([tv, tv]), tri_mat=np.array([0, 0, 1, 1]))
    swap = synth.merge_static(base, np.concatenate([tv, tv]), tri_mat=np.array([1, 1, 0, 0]))
    sun = synth.random_dirs(97)[0]
    a = oracle.eval_srp(both.with_mats(mats), sun, 30, record=True, use_bvh=False)
    b = oracle.eval_srp(swap.with_mats(mats), sun, 30, record=True, use_bvh=False)
    only0 = oracle.eval_srp(base.with_mats(mats[:1]), sun, 30)
    only1 = oracle.eval_srp(base.with_mats(mats[1:]), sun, 30)
    hit = a.ids[:, 0] >= 0
    assert hit.sum() > 0 and (a.ids[hit, 0] <= 1).all()
    np.testing.assert_array_equal(a.force, only0.force)
    np.testing.assert_array_equal(b.force, only1.force)


def test_dihedral_chain_gradient_closed_form():
    """Differentiating the two-hit dihedral closed form (B = 1) in the
    coefficients: dF/drs = sqrt2 L H P (2 rs + (sqrt2/3) rd) d and
    dF/drd = sqrt2 L H P (sqrt2/3)(1 + rs) d.  The weight of the second hit
    carries rs, so this pins the chain term of the fixed-visibility gradient."""
    rs, rd, L, H, P = 0.45, 0.3, 1.1, 0.8, 1.3
    sc = synth.dihedral(L, H, (rs, rd))
    sun = np.array([0.0, 1.0, 1.0]) / np.sqrt(2)
    d = -sun
    r = oracle.eval_srp(sc, sun, 20, bounces=1, pressure=P, record=True)
    g = oracle.fd_gradients(sc, sun, 20, 1, r.grid, r.ids, pressure=P, which=("rho_s", "rho_d"))
    A = np.sqrt(2) * L * H
    np.testing.assert_allclose(g["rho_s"][0], A * P * (2 * rs + np.sqrt(2) / 3 * rd) * d,
                               rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(g["rho_d"][0], A * P * np.sqrt(2) / 3 * (1 + rs) * d,
                               rtol=1e-8, atol=1e-10)


def _dihedral_chains(rho_a, rho_b):
    """The dihedral's two ray families written out by hand (d0 = -(0,1,1)/sqrt2,
    face A in z = 0 with n_A = +z and material rho_a, face B in y = 0 with
    n_B = +y and material rho_b, both normals facing the rays, c = 1/sqrt2 at
    every hit).  Family A hits A first, reflects along R_A d0 = (0,-1,1)/sqrt2
    onto B at the mirrored point; family B likewise.  With
    law(d, n, rs, rd) = (1-rs) d - 2 (rs c(d) + rd/3) n, c(d) = -n.d, the
    per-unit-weight terms of each family's two hits are
        A1 = law(d0, n_A, rho_a),  A2 = rs_a law(R_A d0, n_B, rho_b),
        B1 = law(d0, n_B, rho_b),  B2 = rs_b law(R_B d0, n_A, rho_a)."""
    nA, nB = np.array([0.0, 0.0, 1.0]), np.array([0.0, 1.0, 0.0])
    d0 = -np.array([0.0, 1.0, 1.0]) / np.sqrt(2)

    def law(d, n, rho):
        rs, rd = rho
        return (1 - rs) * d - 2 * (rs * (-(n @ d)) + rd / 3) * n

    RA, RB = np.eye(3) - 2 * np.outer(nA, nA), np.eye(3) - 2 * np.outer(nB, nB)
    return dict(nA=nA, nB=nB, d0=d0, RA=RA, RB=RB,
                A1=law(d0, nA, rho_a), A2=rho_a[0] * law(RA @ d0, nB, rho_b),
                B1=law(d0, nB, rho_b), B2=rho_b[0] * law(RB @ d0, nA, rho_a))


@pytest.mark.parametrize("bounces", [0, 1, 2])
def test_dihedral_torque_off_axis(bounces):
    """Torque of both hits about an off-axis point, faces of different
    materials (so the two families do not mirror each other).  Each family
    covers half the window (N even: the faces' projections meet on a pixel
    edge), so each carries P W/2, W = sqrt2 L H.  Family A's primary hits are
    spread evenly over face A (mean = its centre c_A = (L/2, H/2, 0)) and its
    secondary hits are their mirror images on face B (mean c_B =
    (L/2, 0, H/2)); family B the other way round.  So
        tau = P W/2 [(c_A - r) x A1 + (c_B - r) x A2 + (c_B - r) x B1 + (c_A - r) x B2]
    (A2 = B2 = 0 without a bounce).  A lever arm taken at the wrong hit, or
    at the primary point for the bounce, fails this."""
    rho_a, rho_b, L, H, P = (0.55, 0.25), (0.2, 0.5), 1.3, 0.7, 1.7
    sc = synth.dihedral(L, H, rho_a, rho_b)
    sun = np.array([0.0, 1.0, 1.0]) / np.sqrt(2)
    ref = np.array([0.3, -0.8, 1.1])
    r = oracle.eval_srp(sc, sun, 40, bounces=bounces, pressure=P, ref=ref)
    ch = _dihedral_chains(rho_a, rho_b)
    cA, cB = np.array([L / 2, H / 2, 0.0]), np.array([L / 2, 0.0, H / 2])
    k = 1.0 if bounces else 0.0
    W = np.sqrt(2) * L * H
    tau = P * W / 2 * (np.cross(cA - ref, ch["A1"]) + k * np.cross(cB - ref, ch["A2"]) +
                       np.cross(cB - ref, ch["B1"]) + k * np.cross(cA - ref, ch["B2"]))
    F = P * W / 2 * (ch["A1"] + k * ch["A2"] + ch["B1"] + k * ch["B2"])
    np.testing.assert_allclose(r.force, F, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r.torque, tau, rtol=1e-11, atol=1e-11 * np.abs(tau).max())


@pytest.mark.parametrize("bounces", [1, 2])
def test_dihedral_direction_jacobian(bounces):
    """dF/dd through the two-hit chain, by hand.  At fixed visibility a ray of
    family A carries (c_A(d)/c) [law(d, n_A, rho_a) + rs_a law(R_A d, n_B, rho_b)]
    per unit P A_pix (its share of face A scales with c_A(d) = -n_A.d), so at d0
        J_A = -(A1 + A2) n_A^T / c + D_a(n_A) + rs_a D_b(n_B) R_A,
    with D(n) = d law/dd = (1-rs) I + 2 rs n n^T for that face's material and
    d(R_A d)/dd = R_A; J_B the same with A and B swapped; J = P W/2 (J_A + J_B).
    The oracle's central differences of its frozen re-shade at moved
    directions must agree.  A reflection taken about the wrong normal, a
    reflected direction not carried to the second hit, or a share factor that
    does not follow d, fails this."""
    rho_a, rho_b, L, H, P = (0.45, 0.3), (0.6, 0.15), 1.1, 0.8, 1.3
    sc = synth.dihedral(L, H, rho_a, rho_b)
    sun = np.array([0.0, 1.0, 1.0]) / np.sqrt(2)
    r = oracle.eval_srp(sc, sun, 20, bounces=bounces, pressure=P, record=True)
    ch = _dihedral_chains(rho_a, rho_b)
    nA, nB, RA, RB = ch["nA"], ch["nB"], ch["RA"], ch["RB"]
    c = 1 / np.sqrt(2)
    I3 = np.eye(3)

    def D(n, rho):
        return (1 - rho[0]) * I3 + 2 * rho[0] * np.outer(n, n)

    JA = -np.outer(ch["A1"] + ch["A2"], nA) / c + D(nA, rho_a) + rho_a[0] * D(nB, rho_b) @ RA
    JB = -np.outer(ch["B1"] + ch["B2"], nB) / c + D(nB, rho_b) + rho_b[0] * D(nA, rho_a) @ RB
    J = P * np.sqrt(2) * L * H / 2 * (JA + JB)
    Jfd = oracle.fd_dir_jacobian(sc, 20, bounces, r.grid, r.ids, pressure=P)
    np.testing.assert_allclose(Jfd, J, rtol=1e-7, atol=1e-8 * np.abs(J).max())


def test_two_axis_joint_by_hand():
    """Two-axis wing (support about y, then fold about x, both through the
    wing root): a panel point moves by R_y(a) R_x(b) about the root; the fold
    is limited to +-45 deg and the support to +-90 deg (clamped)."""
    bw = synth.box_wing_2axis()
    ang = np.array([0.7, -0.4, -0.3, 0.5])
    X = oracle.node_transforms(bw, ang)
    p = np.array([0.3, 4.0, 0.1])
    for node, (a, b), piv in ((1, ang[:2], np.array([0, 1.5, 0])), (2, ang[2:], np.array([0, -1.5, 0]))):
        np.testing.assert_allclose(X[node, :, :3] @ p + X[node, :, 3], _Ry(a) @ (_Rx(b) @ (p - piv)) + piv, atol=1e-14)
    np.testing.assert_allclose(oracle.node_transforms(bw, [2.0, 1.5, -3.0, -0.9]),
                               oracle.node_transforms(bw, [np.pi / 2, np.pi / 4, -np.pi / 2, -np.pi / 4]), atol=0)


def test_two_axis_tracking_faces_the_sun():
    """With a support and a fold axis, tracking outer to inner turns the
    panel normal exactly onto the Sun (either face) whenever neither limit
    binds; otherwise the result sits on a limit."""
    from oracle import propagate as OP
    bw = synth.box_wing_2axis()
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(200):
        s = rng.normal(size=3)
        s /= np.linalg.norm(s)
        ang = OP.sun_tracking(bw, s, np.zeros(4))
        for node, j in ((1, 0), (2, 2)):
            n = oracle.node_transforms(bw, ang)[node][:, :3] @ np.array([0.0, 0.0, 1.0])
            inside = abs(ang[j]) < np.pi / 2 - 1e-9 and abs(ang[j + 1]) < np.pi / 4 - 1e-9
            if inside:
                assert abs(abs(n @ s) - 1) < 1e-12
                checked += 1
            else:
                assert np.isclose(abs(ang[j]), np.pi / 2) or np.isclose(abs(ang[j + 1]), np.pi / 4)
    assert checked > 50


def test_frozen_direction_reshade_and_plate_jacobian():
    """The frozen re-shade at a new photon direction gives back the recorded
    force at the recorded direction; for a plate that fills its window (every
    pixel hits, visible share 1) it is F(d) = P A c(d) L(d) with c = -n.d and
    L = (1-rs) d - 2 (rs c + rd/3) n, whose Jacobian by hand is
    dF/dd = P A [-L n^T + c ((1-rs) I + 2 rs n n^T)]."""
    rs, rd, P = 0.35, 0.25, 1.7
    sun = np.array([0.3, -0.2, 1.0])
    sc, d, u, v = _aligned_plate(sun, 2.0, 1.5, 0.6, (rs, rd))
    r = oracle.eval_srp(sc, sun, 32, bounces=1, pressure=P, record=True)
    fr = oracle.shade_frozen(sc, sun, 32, 1, r.grid, r.ids, pressure=P)
    np.testing.assert_allclose(oracle.shade_frozen_dir(sc, 32, 1, r.grid, r.ids, r.grid["d"], pressure=P), fr.force,
                               rtol=1e-12)
    W = sc.verts[sc.tris[0]]
    n = np.cross(W[1] - W[0], W[2] - W[0])
    n /= np.linalg.norm(n)
    if n @ d > 0:
        n = -n
    c = -n @ d
    A = 2.0 * 1.5
    L = (1 - rs) * d - 2 * (rs * c + rd / 3) * n
    np.testing.assert_allclose(r.force, P * A * c * L, rtol=1e-12)
    J = P * A * (-np.outer(L, n) + c * ((1 - rs) * np.eye(3) + 2 * rs * np.outer(n, n)))
    Jfd = oracle.fd_dir_jacobian(sc, 32, 1, r.grid, r.ids, pressure=P)
    np.testing.assert_allclose(Jfd, J, rtol=1e-7, atol=1e-9 * np.abs(J).max())
