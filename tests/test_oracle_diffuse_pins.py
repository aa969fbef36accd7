"""Pins of the oracle's diffuse secondary rays against closed forms and
invariants.

The paper fixes the ray budget (Sec. 6.1: 16 diffuse rays with two levels of
secondary reflections; Sec. 4.3: the secondary rays made at each interaction
set the level of scattering) but not the directions.  The oracle's reading: a
chain hit of generation g < B on a material with rho_d > 0 emits K rays of
weight w rho_d / K along a fixed cosine-weighted direction set; the emitter's
diffuse recoil is the set's mean direction m instead of 2/3 n; a diffuse ray
deposits at its first hit by the flat-plate law and spawns nothing.

The pins hold for any cosine-distributed set as K grows, so they check the
distribution, the weights, the recoil, the transport and the law at the
receiving face without retyping the set:
  * a lone plate is convex, every diffuse ray escapes, and the force tends to
    the Lambertian law (2/3 n recoil) as K grows;
  * in a right-angled corner whose faces are much larger than the distance
    from the hit to the corner line, the other face fills exactly half of the
    emitting face's hemisphere.  With a = 2/(3 pi), the cosine-weighted
    moments over that half are E[omega; omega.m < 0] = -a m_hat + n/3 (m_hat the
    other face's outward normal), E[-omega.m_hat; ...] = a and the probability
    1/2, so the momentum the fan leaves on the other face has a closed form.
"""
import numpy as np
import pytest

import oracle
import synth

A = 2.0 / (3.0 * np.pi)


def _law(w, d, n, rs, rd):
    c = -float(np.dot(n, d))
    return w * ((1 - rs) * d - 2 * (rs * c + rd / 3) * n)


def test_set_is_a_cosine_weighted_unit_set():
    """Every direction is a unit vector in the upper hemisphere; the set's
    mean tends to (0, 0, 2/3) and its second moments to those of the cosine
    distribution (E[l_z^2] = 1/2, E[l_x^2] = E[l_y^2] = 1/4)."""
    for K in (1, 16, 1000):
        L = oracle.diffuse_set(K)
        np.testing.assert_allclose(np.linalg.norm(L, axis=1), 1.0, rtol=0, atol=1e-15)
        assert (L[:, 2] > 0).all()
    L = oracle.diffuse_set(20000)
    np.testing.assert_allclose(L.mean(0), [0, 0, 2 / 3], atol=2e-4)
    np.testing.assert_allclose((L * L).mean(0), [0.25, 0.25, 0.5], atol=2e-4)
    # a uniform hemisphere set would have mean 1/2: the check above tells them apart


@pytest.mark.parametrize("rho", [(0.0, 1.0), (0.3, 0.5)])
def test_lone_plate_tends_to_lambert_recoil(rho):
    """Face-on unit plate (d = -n, c = 1), all diffuse rays escape: the force
    per unit projected area is (1 - rs) d - 2 rs n - rd m, which tends to the
    flat-plate law as K grows; no diffuse ray hits; K rays per primary hit."""
    rs, rd = rho
    sc = synth.plate((0, 0, 0), (1, 0, 0), (0, 1, 0), rho=rho)
    n_pix, prev = 64, None
    for K in (16, 256, 4096):
        r = oracle.eval_srp(sc, (0, 0, 1), n_pix, bounces=1, diffuse=K)
        A_proj = r.grid["a_pix"] * r.n_hits
        assert r.n_hits == n_pix * n_pix
        assert r.n_diffuse == K * r.n_hits and r.n_diffuse_hits == 0
        F = _law(A_proj, np.array([0, 0, -1.0]), np.array([0, 0, 1.0]), rs, rd)
        err = np.linalg.norm(r.force - F) / np.linalg.norm(F)
        if prev is not None:
            assert err < prev or err < 1e-9
        prev = err
    assert prev < 1e-4


@pytest.mark.parametrize("K", [1, 3, 16])
def test_recoil_is_the_exact_mean_of_the_fan(K):
    """At any K the emitter's diffuse recoil is the mean m of its K emitted
    directions, so momentum is accounted for exactly.  Face-on plate, rho_s = 0,
    rho_d = 0.6: F = P A [d - rd m].  The normal component of m is the mean
    of the set's local z components and the length of its tangential part is
    that of the mean of the local (x, y) components; both do not depend on
    how the set is turned about n."""
    rd = 0.6
    sc = synth.plate((0, 0, 0), (1, 0, 0), (0, 1, 0), rho=(0.0, rd))
    r = oracle.eval_srp(sc, (0, 0, 1), 8, bounces=1, diffuse=K)
    PA = r.grid["a_pix"] * r.n_hits
    L = oracle.diffuse_set(K)
    m = L.mean(0)
    np.testing.assert_allclose(r.force[2], -PA * (1 + rd * m[2]), rtol=1e-13)
    np.testing.assert_allclose(np.hypot(r.force[0], r.force[1]), PA * rd * np.hypot(m[0], m[1]),
                               rtol=1e-12, atol=1e-15)


def _corner_pixels(mesh, sun, n, x0, y_range, count, seed):
    """Pixels whose rays reach the floor z = 0 near (x0, y) for y in y_range."""
    g = oracle.grid_of(mesh, sun, n)
    rng = np.random.default_rng(seed)
    pts = np.stack([x0 + rng.uniform(-0.5, 0.5, count), rng.uniform(*y_range, count), np.zeros(count)], 1)
    a, b = pts @ g["u"], pts @ g["v"]
    i = np.floor((a - g["umin"]) / g["wu"] * n).astype(np.int64)
    j = np.floor((b - g["vmin"]) / g["wv"] * n).astype(np.int64)
    return j * n + i


@pytest.mark.parametrize("rho", [(0.0, 1.0), (0.4, 0.5), (0.7, 0.2)])
def test_corner_closed_form(rho):
    """Right-angled corner with faces 2e4 (along x) by 1e4: floor z = 0
    (n_f = +z) and wall y = 0 (n_w = +y), one material.  The Sun at 45 deg in
    the y-z plane: d = (0, -1, -1)/sqrt2 hits the floor (c = 1/sqrt2), the
    specular ray (0, -1, 1)/sqrt2 hits the wall with weight rs, and the next
    one (0, 1, 1)/sqrt2 escapes.  With B = 2 both hits emit fans.  Per unit
    projected area, as K grows:
      floor hit   (1-rs) d - 2 rs c n_f - rd (2/3) n_f
      floor fan   rd [(1-rs)(0, -a, 1/3) - 2 rs a n_w - (rd/3) n_w]   (on the wall)
      wall hit    rs [(1-rs) d' - 2 rs c n_w - rd (2/3) n_w]
      wall fan    rs rd [(1-rs)(0, 1/3, -a) - 2 rs a n_f - (rd/3) n_f] (on the floor)
    Rays start within 1.5 of the corner line, so the faces' finite size changes
    the result by about 1e-4."""
    rs, rd = rho
    mesh = synth.dihedral(L=2e4, H=1e4, rho=rho)
    s2 = np.sqrt(0.5)
    sun = np.array([0.0, s2, s2])
    d, d1 = np.array([0.0, -s2, -s2]), np.array([0.0, -s2, s2])
    nf, nw = np.array([0.0, 0.0, 1.0]), np.array([0.0, 1.0, 0.0])
    per = (_law(1.0, d, nf, rs, rd)
           + rd * ((1 - rs) * np.array([0, -A, 1 / 3]) - 2 * rs * A * nw - rd / 3 * nw)
           + _law(rs, d1, nw, rs, rd)
           + rs * rd * ((1 - rs) * np.array([0, 1 / 3, -A]) - 2 * rs * A * nf - rd / 3 * nf))
    n = 1 << 21
    pix = _corner_pixels(mesh, sun, n, 1e4, (0.5, 1.5), 12, seed=3)
    errs = []
    for K in (64, 8192):
        r = oracle.eval_srp(mesh, sun, n, bounces=2, pixels=pix, diffuse=K, use_bvh=False, record=True)
        assert r.n_hits == len(pix)
        # every ray takes floor -> wall; floor fans land on the wall (triangles 2, 3)
        # or escape, wall fans land on the floor (0, 1) or escape
        assert np.isin(r.ids[:, 0], [0, 1]).all()
        if rs > 0:
            assert np.isin(r.ids[:, 1], [2, 3]).all() and (r.ids[:, 2] == -1).all()
        fan0 = r.ids[:, 3:3 + K]
        fan1 = r.ids[:, 3 + K:3 + 2 * K]
        assert np.isin(fan0, [-1, 2, 3]).all() and np.isin(fan1, [-1, 0, 1]).all()
        assert (fan1 == -1).all() if rs == 0 else True
        F = per * r.grid["a_pix"] * len(pix)
        errs.append(np.linalg.norm(r.force - F) / np.linalg.norm(F))
        # half of each fan hits the other face
        assert abs((fan0 >= 0).mean() - 0.5) < (0.05 if K == 64 else 2e-3)
    assert errs[1] < 2e-4, errs
    assert errs[1] < errs[0]


def test_no_diffuse_material_or_no_secondary_level_changes_nothing():
    """K has no effect when no material has rho_d > 0 or when B = 0 (a fan
    needs a further secondary level): the results are bitwise those of K = 0."""
    sc = synth.procedural_sized(7, 3000)
    sun = synth.random_dirs(5)[0]
    ang = np.linspace(-0.5, 0.5, sc.n_dof)
    nod = sc.with_mats(np.column_stack([sc.mats[:, 0], np.zeros(sc.n_mats)]))
    a = oracle.eval_srp(nod, sun, 48, bounces=2, angles=ang)
    b = oracle.eval_srp(nod, sun, 48, bounces=2, angles=ang, diffuse=16)
    assert a.force.tobytes() == b.force.tobytes() and b.n_diffuse == 0
    a = oracle.eval_srp(sc, sun, 48, bounces=0, angles=ang)
    b = oracle.eval_srp(sc, sun, 48, bounces=0, angles=ang, diffuse=16)
    assert a.force.tobytes() == b.force.tobytes() and b.n_diffuse == 0


def test_fan_counts_and_record_layout():
    """Every chain hit of generation < B on a material with rho_d > 0 emits
    exactly K rays; the record holds B + 1 chain slots then B fans of K."""
    sc = synth.procedural_sized(7, 3000)
    sun = synth.random_dirs(6)[0]
    K, B = 5, 2
    r = oracle.eval_srp(sc, sun, 40, bounces=B, diffuse=K, record=True)
    assert r.ids.shape == (40 * 40, B + 1 + B * K)
    chain = r.ids[:, :B + 1]
    emit = 0
    for g in range(B):
        hit = chain[:, g] >= 0
        rd = np.where(hit, sc.mats[sc.tri_mat[np.maximum(chain[:, g], 0)], 1], 0.0)
        fan = r.ids[:, B + 1 + g * K:B + 1 + (g + 1) * K]
        assert (fan[rd == 0] == -1).all()
        emit += int((rd > 0).sum())
    assert r.n_diffuse == K * emit
    assert r.n_diffuse_hits == int((r.ids[:, B + 1:] >= 0).sum())
    spec = int((chain[:, 1:] >= 0).sum())
    assert r.n_secondary_hits == spec + r.n_diffuse_hits


def test_frozen_shade_reproduces_eval_with_fans():
    """Re-shading the recorded chains and fans at the recording state gives
    back the traced force."""
    sc = synth.procedural_sized(10, 4000)
    ang = np.linspace(-0.8, 0.8, sc.n_dof)
    sun = synth.random_dirs(92)[0]
    r = oracle.eval_srp(sc, sun, 48, bounces=2, angles=ang, record=True, pressure=2.5, diffuse=6)
    assert r.n_diffuse_hits > 0
    s = oracle.shade_frozen(sc, sun, 48, 2, r.grid, r.ids, pressure=2.5, angles=ang, diffuse=6)
    np.testing.assert_allclose(s.force, r.force, rtol=1e-10)
    np.testing.assert_allclose(s.torque, r.torque, rtol=1e-9)
    assert s.n_diffuse_hits == r.n_diffuse_hits and s.n_diffuse == r.n_diffuse
