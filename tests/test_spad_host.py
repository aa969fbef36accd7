"""The library's SPAD interpolation and SPAD propagation (host code, no GPU
needed) against the FP64 oracle's, on the same tables: random tables on the
paper's 20 x 10 grids (plain and shifted by 5 deg, Sec. 6.1), a non-periodic
grid, the poles and the seam; propagation on the paper's orbits; bad inputs."""
import numpy as np
import pytest

from oracle import spad as OS

DEG = np.pi / 180
AU = 1.495978707e11
MU = 1.32712440018e20

GRIDS = [(20, 10, -180 * DEG, -90 * DEG, 18 * DEG, 18 * DEG),
         (20, 10, -175 * DEG, -85 * DEG, 18 * DEG, 18 * DEG),
         (7, 4, -1.0, -0.6, 0.3, 0.35),
         (1, 1, 0.0, 0.0, 1.0, 1.0),
         (36, 1, -np.pi, 0.0, 10 * DEG, 1.0)]


@pytest.fixture(scope="module")
def srp():
    import paper_2608_07307_amd as m
    from paper_2608_07307_amd import _lib as L
    L.load()
    return m


@pytest.mark.parametrize("g", GRIDS)
def test_interp_matches_oracle(srp, g):
    rng = np.random.default_rng(31)
    tab = rng.normal(size=(g[1], g[0], 6)) * 1e-4
    G = srp.spad_grid(*g)
    dirs = [rng.normal(size=3) for _ in range(300)]
    dirs += [np.array(v, float) for v in ((0, 0, 1), (0, 0, -1), (-1, 0, 0), (-1, -1e-17, 0), (-1, 1e-17, 0),
                                          (1, 0, 0), (0, 1, 1e-9))]
    for s in dirs:
        np.testing.assert_allclose(srp.spad_interp(G, tab, s), OS.interp(g, tab, s), rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("orbit", [(0.388, 0.0), (0.388, 0.881), (0.557, 0.682)])
def test_spad_propagation_matches_oracle(srp, orbit):
    """Paper orbits C, E(S), E(L) (Sec. 6.1 table), a quarter period from
    perihelion with a random table on the shifted grid."""
    a, e = orbit[0] * AU, orbit[1]
    rp = a * (1 - e)
    y0 = np.array([rp, 0, 0, 0, np.sqrt(MU * (1 + e) / rp), 0])
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)
    g = GRIDS[1]
    tab = np.random.default_rng(32).normal(size=(10, 20, 6)) * 2e-4
    args = (1.3, y0, 0.0, T / 4 / 200, 200, MU, 800.0, 4.56e-6, AU)
    tr = srp.propagate_spad(srp.spad_grid(*g), tab, *args)
    ref = OS.propagate(g, tab, *args)
    np.testing.assert_allclose(tr[:, 1:4], ref[:, 1:4], rtol=1e-12, atol=1e-2)
    np.testing.assert_allclose(tr[:, 4:], ref[:, 4:], rtol=1e-11, atol=1e-9)


def test_bad_inputs(srp):
    from paper_2608_07307_amd import SrpError
    tab = np.zeros((10, 20, 6))
    for bad in ((0, 10, 0, 0, 0.1, 0.1), (20, 10, 0, 0, 0.0, 0.1), (20, 10, np.nan, 0, 0.1, 0.1),
                (20, 10, 0, 0, 0.1, -1.0)):
        with pytest.raises(SrpError):
            srp.spad_interp(srp.spad_grid(*bad), tab, (1, 0, 0))
    with pytest.raises(SrpError):
        srp.spad_interp(srp.spad_grid(*GRIDS[0]), tab, (0, 0, 0))
    with pytest.raises(SrpError):
        srp.propagate_spad(srp.spad_grid(*GRIDS[0]), tab, 0.0, np.array([AU, 0, 0, 0, 3e4, 0]), 0.0, 60.0, 2,
                           MU, 100.0, 4.56e-6, AU)
