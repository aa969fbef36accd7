"""Articulation slots built on the GPU (one per distinct angle vector of a
batch) against the host's build of the same slot (srp_set_panel_angles):
both compose the node transforms in FP64 from the same cosines and sines and
refit the same top-level topology, so results, test counts and gradients
must be bitwise equal (Sec. 4.4.2 steps 1, 4, 5); every result reports how
many of its angles were clamped to their intervals."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srp():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_07307_amd as m
    return m


MAKERS = {
    "box_wing": lambda: synth.box_wing(),
    "box_wing_2axis": lambda: synth.box_wing_2axis(tess=3),
    "procedural_4k": lambda: synth.procedural_sized(31, 4000),
    # 65 nodes, 64 hinge DOF: four 16-segment wings folding at every joint
    "greebled_small": lambda: synth.greebled_spacecraft(seed=9, bus_n=6, n_greebles=40, seg_nx=2, seg_ny=3),
}


def _dof_limits(mesh):
    lo, hi = [], []
    for k in range(mesh.n_nodes):
        for a in range(int(mesh.n_axes[k])):
            lo.append(mesh.lo[k, a])
            hi.append(mesh.hi[k, a])
    return np.array(lo), np.array(hi)


def _angle_set(mesh, E, seed):
    """E angle vectors: uniform over each interval widened by 0.4 rad (so
    some clamp), a repeat (shares its slot), all zeros and all negative
    zeros (equal angles, distinct bits: distinct slots)."""
    rng = np.random.default_rng(seed)
    lo, hi = _dof_limits(mesh)
    a = rng.uniform(lo - 0.4, hi + 0.4, size=(E, mesh.n_dof))
    a[3] = a[1]
    a[4] = 0.0
    a[5] = -0.0
    return a


@pytest.mark.parametrize("name", list(MAKERS))
def test_device_slots_equal_host_slots(srp, name):
    mesh = MAKERS[name]()
    sc = srp.Scene(mesh)
    E, n, B = 12, 80, 1
    angs = _angle_set(mesh, E, 400 + len(name))
    suns = synth.random_dirs(5100 + len(name), E)
    entries = [(sc, angs[k], srp.params(suns[k], n, B, count=True)) for k in range(E)]
    print(f"{name}: {mesh.n_tris} tris, {mesh.n_nodes} nodes, {mesh.n_dof} DOF, {E} items", flush=True)
    out = srp.results_to_numpy(srp.eval_batch(entries))
    fields = ("force", "torque", "n_rays", "n_hits", "n_secondary", "n_secondary_hits", "n_box_tests",
              "n_tri_tests", "status", "n_clamped")
    lo, hi = _dof_limits(mesh)
    for k in range(E):
        n_clamped = sc.set_angles(angs[k])
        assert n_clamped == int(((angs[k] < lo) | (angs[k] > hi)).sum()), (name, k)
        s = srp.eval(sc, suns[k], n, bounces=B, count=True)
        assert s["n_clamped"] == n_clamped, (name, k)
        for f in fields:
            assert np.array_equal(np.asarray(out[k][f]), np.asarray(s[f])), (name, k, f, out[k][f], s[f])
    assert out[0]["n_hits"] > 0
    assert out["n_clamped"].max() > 0
    # gradients (world hinge axes and transforms of the slot enter them); the
    # single evaluation always returns the photon-direction Jacobian too
    gentries = [(sc, angs[k], srp.params(suns[k], n, B, grad_dir=True)) for k in range(E)]
    _, grad = srp.eval_grad_batch(gentries)
    g = grad.cpu().numpy()
    M, J = mesh.n_mats, mesh.n_dof
    for k in (0, 2, 3, 5, E - 1):
        sc.set_angles(angs[k])
        s = srp.eval_grad(sc, suns[k], n, bounces=B)
        row = np.concatenate([s["rho_s"].ravel(), s["rho_d"].ravel(), s["theta"].ravel(), s["dir"].ravel()])
        assert row.tobytes() == g[k, : 3 * (2 * M + J) + 9].tobytes(), (name, k)
