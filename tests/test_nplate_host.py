"""The library's N-plate force and N-plate propagation (host code, no GPU
needed) against the FP64 oracle's on the same plates: random plate sets,
RK4 and RK7(8) propagation on the paper's orbits (Sec. 6.1 table), bad
inputs."""
import numpy as np
import pytest

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
