"""GPU parity at the benchmark workloads' full sizes, through the same batched
C-ABI calls the benchmark times: sampled items against the FP64 oracle (one
evaluation at a time), properties that hold at any size for the rest, and the
deep-hierarchy case that takes the traversal stack past its LDS part."""
import numpy as np
import pytest

import oracle
import synth
from parity import G_TOL_VM, check_grads, check_report, classify_primary, compare_eval, grad_report, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srp():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_07307_amd as m
    return m


def _entries(srp, scene, dirs, angles, n, bounces):
    return [(scene, angles[k], srp.params(dirs[k], n, bounces)) for k in range(len(dirs))]


def _check_item(srp, tag, scene, mesh, sun, n, bounces, ang, got):
    """One batch item: its single recorded evaluation (the GPU's per-pixel
    hits) gives bitwise the batch result; against the oracle's evaluation with
    the edge-band policy (ids outside the band equal, visibility-matched force
    and torque within F_TOL, plain force within what flipped rays carry).
    Returns the oracle's recorded evaluation and the GPU's."""
    scene.set_angles(ang)
    single = srp.eval(scene, sun, n, bounces=bounces, record=True)
    assert np.array_equal(single["force"], got["force"]) and np.array_equal(single["torque"], got["torque"])
    o = oracle.eval_srp(mesh, sun, n, bounces=bounces, angles=ang, record=True)
    rep = compare_eval(mesh, ang, sun, n, bounces, single, o)
    print(f"{tag}:", {k: (round(v, 9) if isinstance(v, float) else v) for k, v in rep.items()}, flush=True)
    check_report(rep)
    return o, single


def _grad_blocks(g, M, J):
    return g[: 3 * M].reshape(M, 3), g[3 * M: 6 * M].reshape(M, 3), g[6 * M: 6 * M + 3 * J].reshape(J, 3)


def _check_grad(tag, mesh, sun, n, bounces, ang, o, single, g, theta_idx=None):
    """Adjoint against FP64 central differences of the oracle's fixed-visibility
    re-shade, each block (rho_s, rho_d, theta) against its own largest entry:
    on the GPU's recorded hits (visibility matched) within G_TOL_VM, on the
    oracle's own recorded hits within G_TOL beyond the share of the rays whose
    hits differ (edge-band flips)."""
    grid = oracle.grid_of(mesh, sun, n, angles=ang)
    gs, gd, gt = _grad_blocks(g, mesh.n_mats, mesh.n_dof)
    got = {"rho_s": gs, "rho_d": gd, "theta": gt}
    rep = grad_report(got, mesh, sun, n, bounces, grid, o.ids, single["ids"], angles=ang, theta_idx=theta_idx)
    print(f"{tag} per-block gradient err (oracle hits, GPU hits, flipped share): {rep}", flush=True)
    check_grads(rep)


def test_c2_benchmark_batch(srp):
    """The benchmark's batch as it is timed (64 attitudes of the ~50k
    spacecraft, 1024^2 rays, 2 bounces, srp_eval_grad_batch): three sampled
    items against the oracle, item 0's gradients against the oracle's finite
    differences, and the forward-only batch bitwise equal to the forward part
    of the adjoint launch."""
    mesh, dirs, angles, n, B = synth.c2_batch(64)
    sc = srp.Scene(mesh)
    entries = _entries(srp, sc, dirs, angles, n, B)
    res, grad = srp.eval_grad_batch(entries)
    r = srp.results_to_numpy(res).copy()
    g = grad.cpu().numpy()
    assert (r["status"] == 0).all() and (r["n_rays"] == n * n).all()
    fwd = srp.results_to_numpy(srp.eval_batch(entries))
    assert fwd["force"].tobytes() == r["force"].tobytes()
    for k in (0, 37, 63):
        o, single = _check_item(srp, f"c2 item {k}", sc, mesh, dirs[k], n, B, angles[k], r[k])
        if k == 0:
            _check_grad("c2 item 0", mesh, dirs[0], n, B, angles[0], o, single, g[0])


def test_c3_spad_table(srp):
    """The SPAD-style table: 4096 Fibonacci directions x 8 root-hinge angles
    (32,768 evaluations at 512^2, 1 bounce) in one call (the library splits it
    into sub-batches within its workspace bound).  Every item succeeds and has
    hits; sampled items agree with the oracle; a re-run of a slice as its own
    batch is bitwise identical."""
    mesh, dirs, angles, n, B = synth.c3_spad()
    sc = srp.Scene(mesh)
    entries = _entries(srp, sc, dirs, angles, n, B)
    r = srp.results_to_numpy(srp.eval_batch(entries)).copy()
    assert len(r) == 32768
    assert (r["status"] == 0).all() and (r["n_hits"] > 0).all() and np.isfinite(r["force"]).all()
    for k in (5, 12345, 32767):
        _check_item(srp, f"c3 item {k}", sc, mesh, dirs[k], n, B, angles[k], r[k])
    part = srp.results_to_numpy(srp.eval_batch(entries[1000:1064]))
    assert part.tobytes() == r[1000:1064].tobytes()


def test_c4_uneven_batch(srp):
    """The uneven batch: 64 scenes of 1k..450k triangles with grids 256..1920
    in one launch, 1 bounce.  The three smallest items against the oracle in
    full; for the largest scene, primary hit ids on 4096 sampled pixels of its
    own evaluation against the oracle's (edge band excepted) and its batch
    result bitwise equal to the single evaluation."""
    items, B = synth.c4_uneven()
    scenes = [srp.Scene(m) for m, _, _, _ in items]
    entries = [(scenes[k], a, srp.params(s, n, B)) for k, (m, a, s, n) in enumerate(items)]
    r = srp.results_to_numpy(srp.eval_batch(entries)).copy()
    assert (r["status"] == 0).all()
    work = [m.n_tris * n * n for m, _, _, n in items]
    for k in np.argsort(work)[:3]:
        m, a, s, n = items[k]
        _check_item(srp, f"c4 item {k} (T={m.n_tris}, N={n})", scenes[k], m, s, n, B, a, r[k])
    big = int(np.argmax([m.n_tris for m, _, _, _ in items]))
    m, a, s, n = items[big]
    scenes[big].set_angles(a)
    single = srp.eval(scenes[big], s, n, bounces=B, record=True)
    assert np.array_equal(single["force"], r[big]["force"])
    pix = np.random.default_rng(44).choice(n * n, 4096, replace=False)
    o = oracle.eval_srp(m, s, n, bounces=B, angles=a, pixels=pix, record=True)
    grid = oracle.grid_of(m, s, n, angles=a)
    ids_gpu = single["ids"][pix]
    same = ids_gpu[:, 0] == o.ids[:, 0]
    print(f"c4 largest item {big} (T={m.n_tris}, N={n}): primary ids equal on {same.mean():.5f} of 4096 pixels",
          flush=True)
    if not same.all():
        full_o = np.full((n * n,), -1, np.int32)
        full_g = np.full((n * n,), -1, np.int32)
        full_o[pix], full_g[pix] = o.ids[:, 0], ids_gpu[:, 0]
        mism, outside, _ = classify_primary(m, a, grid, n, full_o, full_g)
        assert outside == 0, (mism, outside)


@pytest.fixture(scope="module")
def c5(srp):
    """The ~1M-triangle, 64-hinge spacecraft: 256 attitudes at 2048^2 with the
    adjoint, one srp_eval_grad_batch call (as the benchmark's C5 line)."""
    mesh, dirs, angles, n, B = synth.c5_batch(256)
    sc = srp.Scene(mesh)
    entries = _entries(srp, sc, dirs, angles, n, B)
    res, grad = srp.eval_grad_batch(entries)
    r = srp.results_to_numpy(res).copy()
    g = grad.cpu().numpy().copy()
    yield mesh, sc, dirs, angles, n, B, r, g
    sc.close()


@pytest.mark.parametrize("k", [17, 101, 166, 230])
def test_c5_adjoint_attitude(srp, c5, k):
    """C5, one of four seeded attitudes: every item of the batch succeeded;
    this item's force against the oracle-traced evaluation, and all 16
    material terms and all 64 hinge derivatives per block against the
    oracle's central differences, on the oracle's hits and on the GPU's."""
    mesh, sc, dirs, angles, n, B, r, g = c5
    assert (r["status"] == 0).all() and np.isfinite(g).all()
    o, single = _check_item(srp, f"c5 item {k}", sc, mesh, dirs[k], n, B, angles[k], r[k])
    _check_grad(f"c5 item {k}", mesh, dirs[k], n, B, angles[k], o, single, g[k])


def test_c5_directional_fd_all_attitudes(srp, c5):
    """C5, every one of the 256 attitudes: the adjoint contracted with a seeded
    random direction v in (rho_s, rho_d, theta) space equals the central
    difference of the oracle's fixed-visibility re-shade of the GPU's own
    recorded hits along v (materials and hinges moved together, h = 1e-4),
    to G_TOL_VM of the contracted gradient's size |v| |grad|."""
    mesh, sc, dirs, angles, n, B, r, g = c5
    M, J = mesh.n_mats, mesh.n_dof
    rng = np.random.default_rng(5005)
    h = 1e-4
    worst = 0.0
    for k in range(len(dirs)):
        sc.set_angles(angles[k])
        single = srp.eval(sc, dirs[k], n, bounces=B, record=True)
        assert np.array_equal(single["force"], r[k]["force"])
        gs, gd, gt = _grad_blocks(g[k], M, J)
        vs, vd, vt = rng.uniform(-1, 1, M), rng.uniform(-1, 1, M), rng.uniform(-1, 1, J)
        pred = vs @ gs + vd @ gd + vt @ gt
        grid = oracle.grid_of(mesh, dirs[k], n, angles=angles[k])
        step = np.stack([vs, vd], 1)
        F = []
        for sgn in (1, -1):
            m = mesh.mats + sgn * h * step
            assert (m >= 0).all() and (m.sum(1) <= 1).all()
            F.append(oracle.shade_frozen(mesh.with_mats(m), dirs[k], n, B, grid, single["ids"],
                                         angles=angles[k] + sgn * h * vt, angles_ref=angles[k]).force)
        fd = (F[0] - F[1]) / (2 * h)
        size = np.sqrt((vs ** 2).sum() + (vd ** 2).sum() + (vt ** 2).sum()) * np.abs(g[k][: 3 * (2 * M + J)]).max()
        err = np.abs(pred - fd).max() / size
        worst = max(worst, err)
        assert err <= G_TOL_VM, (k, pred, fd, err)
    print(f"c5 directional FD over 256 attitudes: worst err / (|v| max|grad|) = {worst:.2e}", flush=True)


def test_deep_hierarchy_spills_the_stack(srp):
    """2^20 stacked plates (2M triangles) seen face-on: every child box on the
    way to the top plate is hit, so the descent pushes three entries per 4-wide
    level (~27), more than the register and the LDS ring hold, and the global
    spill path runs.  The force equals the face-on plate closed form
    P*A*(1 + rho_s + 2 rho_d / 3) along the photon direction; every ray hits
    the top plate, as in the oracle."""
    mesh = synth.stacked_plates(1 << 20)
    sc = srp.Scene(mesh)
    rs, rd = mesh.mats[0]
    g = srp.eval(sc, (0, 0, 1), 32, bounces=1, pressure=1.5, record=True)
    F = 1.5 * 1.0 * (1 + rs + 2 * rd / 3) * np.array([0.0, 0.0, -1.0])
    print(f"stacked plates: F {g['force']} closed form {F}, hits {g['n_hits']}", flush=True)
    assert g["n_hits"] == 32 * 32 and rel(g["force"], F) < 1e-6
    o = oracle.eval_srp(mesh, (0, 0, 1), 32, bounces=1, pressure=1.5, record=True)
    # every ray hits the top plate (triangles 2p and 2p + 1 form plate p); which
    # of its two triangles a ray on the shared diagonal reports is a tie
    top = (1 << 20) - 1
    assert (g["ids"][:, 0] // 2 == top).all() and (o.ids[:, 0] // 2 == top).all()
    b = srp.results_to_numpy(srp.eval_batch([(sc, None, srp.params((0, 0, 1), 32, 1, 1.5))]))
    assert np.array_equal(b[0]["force"], g["force"])
