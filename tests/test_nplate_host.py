"""The library's N-plate model (host code, no GPU needed) against the FP64
oracle's: the plates it derives from a mesh (triangles merged per node,
material and normal, moved with the hinges) against one plate per triangle,
the force on random plate sets, RK4 and RK7(8) propagation on the paper's
orbits (Sec. 6.1 table), bad inputs."""
import numpy as np
import pytest

import synth
from oracle import nplate as NP

AU = 1.495978707e11
MU = 1.32712440018e20
P1AU = 4.56e-6


@pytest.fixture(scope="module")
def srp():
    import paper_2608_07307_amd as m
    from paper_2608_07307_amd import _lib as L
    L.load()
    return m


def _random_plates(seed, n):
    rng = np.random.default_rng(seed)
    p = np.zeros(n, NP.PLATE_DTYPE)
    nv = rng.normal(size=(n, 3))
    p["normal"] = nv / np.linalg.norm(nv, axis=1)[:, None]
    p["center"] = rng.uniform(-3, 3, size=(n, 3))
    p["area"] = rng.uniform(0.01, 4.0, size=n)
    p["rho_s"] = rng.uniform(0, 0.6, size=n)
    p["rho_d"] = rng.uniform(0, 0.3, size=n)
    p["two_sided"] = rng.integers(0, 2, size=n)
    return p


def test_force_matches_oracle(srp):
    pl = _random_plates(51, 60)
    rng = np.random.default_rng(52)
    for k in range(25):
        s = rng.normal(size=3) * rng.uniform(0.1, 10)
        ref = rng.uniform(-1, 1, size=3)
        P = rng.uniform(1e-7, 1e-4)
        got = srp.nplate_eval(pl, s, P, ref)
        F, T = NP.force(pl, s, P, ref)
        np.testing.assert_allclose(got["force"], F, rtol=1e-12, atol=1e-12 * np.abs(F).max())
        np.testing.assert_allclose(got["torque"], T, rtol=1e-12, atol=1e-12 * np.abs(T).max())
    empty = srp.nplate_eval(np.zeros(0, srp.PLATE_DTYPE), (1, 0, 0), 1.0)
    assert np.all(empty["force"] == 0) and np.all(empty["torque"] == 0)


@pytest.mark.parametrize("orbit", [(0.388, 0.0), (0.557, 0.682)])
def test_propagation_matches_oracle(srp, orbit):
    """RK4 and fixed-step RK7(8) over a quarter period from perihelion."""
    a, e = orbit[0] * AU, orbit[1]
    rp = a * (1 - e)
    y0 = np.array([rp, 0, 0, 0, np.sqrt(MU * (1 + e) / rp), 0])
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)
    pl = _random_plates(53, 20)
    args = (MU, 50.0, P1AU, AU)
    tr = srp.propagate_nplate(pl, y0, 0.0, T / 4 / 100, 100, *args)
    ref = NP.propagate(pl, y0, 0.0, T / 4 / 100, 100, *args)
    np.testing.assert_allclose(tr[:, 1:4], ref[:, 1:4], rtol=1e-12, atol=1e-2)
    np.testing.assert_allclose(tr[:, 4:], ref[:, 4:], rtol=1e-11, atol=1e-9)
    opts = srp.rk78_opts(T / 4 / 40)
    tr8 = srp.propagate_nplate_rk78(pl, y0, 0.0, T / 4, opts, *args)
    ref8, _ = NP.propagate_rk78(pl, y0, 0.0, T / 4, T / 4 / 40, *args)
    assert tr8.shape == ref8.shape
    np.testing.assert_allclose(tr8[:, 1:4], ref8[:, 1:4], rtol=1e-12, atol=1e-2)
    np.testing.assert_allclose(tr8[:, 4:], ref8[:, 4:], rtol=1e-11, atol=1e-9)


def test_bad_inputs(srp):
    from paper_2608_07307_amd import SrpError
    good = _random_plates(54, 3)
    for field, value in (("area", 0.0), ("area", -1.0), ("rho_s", 1.5), ("rho_d", -0.1)):
        bad = good.copy()
        bad[field][1] = value
        with pytest.raises(SrpError):
            srp.nplate_eval(bad, (1, 0, 0), 1.0)
    bad = good.copy()
    bad["normal"][0] = (1.0, 1.0, 0.0)
    with pytest.raises(SrpError):
        srp.nplate_eval(bad, (1, 0, 0), 1.0)
    with pytest.raises(SrpError):
        srp.nplate_eval(good, (0, 0, 0), 1.0)
    with pytest.raises(SrpError):
        srp.propagate_nplate(good, np.array([AU, 0, 0, 0, 3e4, 0]), 0.0, 60.0, 2, MU, 0.0, P1AU, AU)


@pytest.mark.parametrize("maker", [synth.box_wing, lambda: synth.box_wing_2axis(tess=3),
                                   lambda: synth.procedural_spacecraft(seed=2)])
def test_plates_from_mesh_match_oracle(srp, maker):
    """Merged plates give the per-triangle model's force and torque (the model
    is linear in the plates; the library's vertices are FP32)."""
    m = maker()
    ang = np.random.default_rng(61).uniform(-0.6, 0.6, size=m.n_dof)
    pl = srp.nplate_from_mesh(m, ang)
    ref = NP.plates(m, ang)
    assert 0 < len(pl) <= len(ref)
    np.testing.assert_allclose(pl["area"].sum(), ref["area"].sum(), rtol=1e-6)
    assert int(pl["two_sided"].any()) == int(ref["two_sided"].any())
    for s in synth.random_dirs(6101, 12):
        F, T = NP.force(ref, s, P1AU, (0.2, -0.1, 0.3))
        got = srp.nplate_eval(pl, s, P1AU, (0.2, -0.1, 0.3))
        f = np.abs(F).max()
        np.testing.assert_allclose(got["force"], F, rtol=2e-6, atol=2e-6 * f)
        np.testing.assert_allclose(got["torque"], T, rtol=2e-6, atol=2e-6 * max(np.abs(T).max(), f))


def test_box_wing_plates_from_mesh(srp):
    """Six bus faces and two two-sided 2 x 5 m panels; the panels turn with
    their hinges (rest normal +z, hinge about y)."""
    pl = srp.nplate_from_mesh(synth.box_wing(), [0.7, -0.4])
    assert len(pl) == 8 and int(pl["two_sided"].sum()) == 2
    np.testing.assert_allclose(np.sort(pl["area"]), [1, 1, 1, 1, 1, 1, 10, 10], rtol=1e-6)
    panels = pl[pl["two_sided"] == 1]
    for th in (0.7, -0.4):
        n = np.array([np.sin(th), 0.0, np.cos(th)])
        assert min(np.abs(np.abs(panels["normal"] @ n) - 1.0)) < 1e-7
    rest = srp.nplate_from_mesh(synth.box_wing())
    np.testing.assert_allclose(np.abs(rest[rest["two_sided"] == 1]["normal"][:, 2]), 1.0, rtol=1e-12)


def test_plates_from_mesh_errors(srp):
    from paper_2608_07307_amd import SrpError
    m = synth.box_wing()
    m.tri_mat = np.array(m.tri_mat).copy()
    m.tri_mat[0] = 99
    with pytest.raises(SrpError):
        srp.nplate_from_mesh(m)


def test_plates_from_mesh_rejects_wrong_angle_count(srp):
    """The library reads n_dof angles: a shorter (or longer) vector is an
    error raised before the call, not an out-of-bounds read."""
    from paper_2608_07307_amd import SrpError
    m = synth.box_wing()
    for bad in ([0.1], [0.1, 0.2, 0.3], np.zeros((1, 1))):
        with pytest.raises(SrpError):
            srp.nplate_from_mesh(m, bad)
    assert len(srp.nplate_from_mesh(m, [0.1, -0.2])) > 0
