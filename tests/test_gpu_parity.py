"""GPU parity: the gfx950 library (through the C ABI) against the FP64 oracle
and against closed forms, on seeded synthetic inputs."""
import numpy as np
import pytest

import oracle
import synth
from parity import F_TOL, compare_eval, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srp():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_07307_amd as m
    return m


def _show(tag, rep):
    print(tag, {k: (round(v, 9) if isinstance(v, float) else v) for k, v in rep.items()}, flush=True)


def _check(rep, strict=True):
    assert rep["primary_outside_band"] == 0, rep
    assert rep["f_err_vis_matched"] <= F_TOL, rep
    assert rep["t_err_vis_matched"] <= F_TOL, rep
    if strict:
        assert rep["f_err"] <= F_TOL, rep
        assert rep["t_err"] <= F_TOL, rep


@pytest.mark.parametrize("seed", [1001, 1002, 1003, 1004])
@pytest.mark.parametrize("angles", [(0.0, 0.0), (0.7, -1.1)])
def test_box_wing_128(srp, seed, angles):
    """Box-wing, 128 x 128 rays, primary hits only (the smallest workload)."""
    mesh = synth.box_wing()
    sc = srp.Scene(mesh)
    sc.set_angles(angles)
    sun = synth.random_dirs(seed)[0]
    g = srp.eval(sc, sun, 128, bounces=0, record=True)
    o = oracle.eval_srp(mesh, sun, 128, bounces=0, angles=angles, record=True)
    rep = compare_eval(mesh, angles, sun, 128, 0, g, o)
    _show(f"box_wing seed={seed} angles={angles}", rep)
    _check(rep)


@pytest.mark.parametrize("bounces", [0, 1, 2])
def test_box_wing_bounces(srp, bounces):
    mesh = synth.box_wing()
    sc = srp.Scene(mesh)
    ang = (0.9, 0.5)
    sc.set_angles(ang)
    for seed in (1011, 1012):
        sun = synth.random_dirs(seed)[0]
        g = srp.eval(sc, sun, 96, bounces=bounces, record=True)
        o = oracle.eval_srp(mesh, sun, 96, bounces=bounces, angles=ang, record=True)
        rep = compare_eval(mesh, ang, sun, 96, bounces, g, o)
        _show(f"box_wing B={bounces} seed={seed}", rep)
        _check(rep)


def test_closed_forms_on_gpu(srp):
    """Face-on cube and the 90-degree dihedral retroreflector on the GPU
    (closed forms derived in test_oracle_pins)."""
    rs, rd = 0.3, 0.25
    sc = srp.Scene(synth.cube(0.75, (rs, rd)))
    g = srp.eval(sc, (0, 0, 1), 64, bounces=1, pressure=2.0)
    F = 2.0 * 1.5 * 1.5 * (1 + rs + 2 * rd / 3) * np.array([0, 0, -1.0])
    assert g["n_hits"] == 64 * 64
    assert rel(g["force"], F) < 1e-6
    L, H = 1.3, 0.7
    for rho in ((1.0, 0.0), (0.5, 0.3)):
        sc = srp.Scene(synth.dihedral(L, H, rho))
        sun = np.array([0.0, 1.0, 1.0]) / np.sqrt(2)
        g = srp.eval(sc, sun, 64, bounces=2, pressure=1.7)
        k = 1 + rho[0] ** 2 + np.sqrt(2) / 3 * (1 + rho[0]) * rho[1]
        F = np.sqrt(2) * L * H * 1.7 * k * (-sun)
        assert g["n_hits"] == 64 * 64 and g["n_secondary_hits"] == 64 * 64
        assert rel(g["force"], F) < 1e-6, (g["force"], F)


def test_procedural_reduced(srp):
    """~50k-triangle procedural spacecraft at 256 x 256 rays, 2 bounces."""
    mesh = synth.procedural_spacecraft()
    sc = srp.Scene(mesh)
    ang = np.linspace(-0.6, 0.6, mesh.n_dof)
    sc.set_angles(ang)
    for seed in (1002, 1005):
        sun = synth.random_dirs(seed)[0]
        g = srp.eval(sc, sun, 256, bounces=2, record=True)
        o = oracle.eval_srp(mesh, sun, 256, bounces=2, angles=ang, record=True)
        rep = compare_eval(mesh, ang, sun, 256, 2, g, o)
        _show(f"procedural 256 B=2 seed={seed}", rep)
        _check(rep)
        assert rep["secondary_match_fraction"] > 0.999
