"""Multi-axis joints on the GPU (Sec. 4.4.1: up to three axes per edge label;
the paper's BoxWing wings turn about a support axis within +-90 deg and fold
within +-45 deg; its PSP arrays move within +-30 deg): evaluations at random
two-axis settings, library sun tracking against the oracle's, a PSP-like
spacecraft whose wing roots are limited to +-30 deg, and a tracking
propagation of the two-axis craft."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import propagate as OP
import synth
from parity import check_report, compare_eval

pytestmark = pytest.mark.gpu

MU = 1.32712440018e20
AU = 1.495978707e11
P0 = 1361.0 / 299792458.0


@pytest.fixture(scope="module")
def srp():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_07307_amd as m
    return m


def test_two_axis_evaluations(srp):
    mesh = synth.box_wing_2axis(tess=4)
    sc = srp.Scene(mesh)
    rng = np.random.default_rng(51)
    for k in range(6):
        ang = rng.uniform(-1, 1, 4) * np.array([1.5, 0.75, 1.5, 0.75])
        sc.set_angles(ang)
        sun = synth.random_dirs(5100 + k)[0]
        g = srp.eval(sc, sun, 96, bounces=2, record=True)
        o = oracle.eval_srp(mesh, sun, 96, bounces=2, angles=ang, record=True)
        rep = compare_eval(mesh, ang, sun, 96, 2, g, o)
        check_report(rep)


def test_two_axis_tracking_matches_oracle(srp):
    mesh = synth.box_wing_2axis()
    sc = srp.Scene(mesh)
    rng = np.random.default_rng(52)
    for k in range(20):
        sun = synth.random_dirs(5200 + k)[0]
        start = rng.uniform(-0.5, 0.5, 4)
        np.testing.assert_allclose(srp.sun_tracking_angles(sc, sun, start), OP.sun_tracking(mesh, sun, start),
                                   rtol=0, atol=1e-12)


def _psp_like():
    """The procedural spacecraft with its wing roots limited to +-30 deg."""
    m = synth.procedural_spacecraft(seed=2, dish_rings=8, dish_sectors=8, seg_nx=4, seg_ny=4)
    lo, hi = m.lo.copy(), m.hi.copy()
    for k in range(1, m.n_nodes):
        if m.is_panel[k] and not m.is_panel[m.parent[k]]:
            lo[k, 0], hi[k, 0] = -np.pi / 6, np.pi / 6
    return dataclasses.replace(m, lo=lo, hi=hi)


def test_limited_wing_roots(srp):
    """Tracking clamps the roots to +-30 deg (library and oracle agree), and the
    clamped articulation evaluates as the oracle's."""
    mesh = _psp_like()
    sc = srp.Scene(mesh)
    roots = [int(np.concatenate([[0], np.cumsum(mesh.n_axes)])[k]) for k in range(1, mesh.n_nodes)
             if mesh.is_panel[k] and not mesh.is_panel[mesh.parent[k]]]
    clamped = 0
    for k in range(8):
        sun = synth.random_dirs(5300 + k)[0]
        a = srp.sun_tracking_angles(sc, sun)
        np.testing.assert_allclose(a, OP.sun_tracking(mesh, sun, np.zeros(mesh.n_dof)), rtol=0, atol=1e-12)
        assert all(abs(a[j]) <= np.pi / 6 + 1e-15 for j in roots)
        clamped += sum(np.isclose(abs(a[j]), np.pi / 6) for j in roots)
        if k < 3:
            sc.set_angles(a)
            g = srp.eval(sc, sun, 128, bounces=1, record=True)
            o = oracle.eval_srp(mesh, sun, 128, bounces=1, angles=a, record=True)
            check_report(compare_eval(mesh, a, sun, 128, 1, g, o))
    assert clamped > 0


def test_two_axis_tracking_propagation(srp):
    """RK4 with sun-tracking two-axis wings (4 DOF) on a 1 AU orbit inclined
    0.3 rad (the Sun leaves the fold-free plane), 6 one-hour steps, against
    the oracle propagator."""
    mesh = synth.box_wing_2axis()
    sc = srp.Scene(mesh)
    v = np.sqrt(MU / AU)
    y0 = np.array([AU, 0.0, 0.0, 0.0, v * np.cos(0.3), v * np.sin(0.3)])
    kw = dict(mu=MU, mass=1000.0, p_ref=P0, r_ref=AU, n=64, bounces=1, track_sun=True)
    tr, st = srp.propagate(sc, y0, 0.0, 3600.0, 6, **kw)
    ref = OP.propagate(mesh, y0, 0.0, 3600.0, 6, **kw)
    kep = OP.rk4(lambda t, y: np.concatenate([y[3:], -MU * y[:3] / np.linalg.norm(y[:3]) ** 3]), y0, 0.0, 3600.0, 6)
    disp = np.linalg.norm(ref[-1, 1:4] - kep[-1, 1:4])
    err = np.linalg.norm(tr[-1, 1:4] - ref[-1, 1:4])
    print(f"two-axis tracking propagation: SRP displacement {disp:.4f} m, GPU-oracle {err:.2e} m", flush=True)
    assert disp > 1.0 and err <= 1e-4 * disp + 1e-4
