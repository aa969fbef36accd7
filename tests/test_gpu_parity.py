"""GPU parity: the gfx950 library (through the C ABI) against the FP64 oracle
and against closed forms, on seeded synthetic inputs."""
import numpy as np
import pytest

import oracle
import synth
from parity import F_TOL, block_err, check_grads, check_report, compare_eval, grad_report, rel

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
    check_report(rep, strict)


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


def test_articulated_equals_prerotated(srp):
    """Instance-transformed panels give the evaluation of the same mesh
    supplied with pre-rotated vertices (the paper's CPU geometry update,
    Sec. 4.4.2 step 5): ids equal outside the edge band, forces to 1e-5."""
    mesh = synth.procedural_sized(21, 6000)
    ang = np.linspace(-1.2, 1.0, mesh.n_dof)
    sc = srp.Scene(mesh)
    sc.set_angles(ang)
    static = synth.merge_static(mesh, oracle.articulate(mesh, ang))
    st = srp.Scene(static)
    for seed in (2101, 2102, 2103):
        sun = synth.random_dirs(seed)[0]
        a = srp.eval(sc, sun, 192, bounces=2, record=True)
        b = srp.eval(st, sun, 192, bounces=2, record=True)
        o = oracle.eval_srp(mesh, sun, 192, bounces=2, angles=ang, record=True)
        rep = compare_eval(mesh, ang, sun, 192, 2, a, o)
        rep_b = compare_eval(static, None, sun, 192, 2, b, o)
        _show(f"articulated seed={seed}", rep)
        _show(f"pre-rotated seed={seed}", rep_b)
        _check(rep)
        _check(rep_b)
        assert rel(a["force"], b["force"]) <= F_TOL


def test_batch_matches_single_and_is_deterministic(srp):
    """A batch with mixed scenes, grid sizes, bounce counts and angles gives
    bitwise the per-item srp_eval results, and repeated runs are bitwise
    identical (fixed-order reduction, no floating-point atomics)."""
    import torch
    m1, m2 = synth.box_wing(), synth.procedural_sized(22, 4000)
    s1, s2 = srp.Scene(m1), srp.Scene(m2)
    entries, singles = [], []
    for k in range(12):
        sc, m = (s1, m1) if k % 3 == 0 else (s2, m2)
        ang = np.full(m.n_dof, 0.1 * (k % 4) - 0.15)
        n = [64, 100, 128, 37][k % 4]
        B = k % 3
        sun = synth.random_dirs(2200 + k)[0]
        entries.append((sc, ang, srp.params(sun, n, B)))
        sc.set_angles(ang)
        singles.append(srp.eval(sc, sun, n, bounces=B))
    out = srp.results_to_numpy(srp.eval_batch(entries))
    out2 = srp.results_to_numpy(srp.eval_batch(entries))
    prebuilt = srp.Batch(entries)   # marshalled once, launched twice
    out3 = srp.results_to_numpy(srp.eval_batch(prebuilt))
    out4 = srp.results_to_numpy(srp.eval_batch(prebuilt))
    torch.cuda.synchronize()
    assert out3.tobytes() == out.tobytes() and out4.tobytes() == out.tobytes()
    for k, s in enumerate(singles):
        assert np.array_equal(out[k]["force"], s["force"]), k
        assert np.array_equal(out[k]["torque"], s["torque"]), k
        assert out[k]["n_hits"] == s["n_hits"] and out[k]["n_secondary_hits"] == s["n_secondary_hits"]
    assert out.tobytes() == out2.tobytes()


def test_back_to_back_batches_on_different_streams(srp):
    """Consecutive launches through the library's shared workspace on three
    streams, with no synchronisation between them: the host prepares each
    launch while the previous one runs and the library orders it after that
    one on the device, so every result (forward and adjoint) is bitwise its
    reference taken alone."""
    import torch
    mesh = synth.procedural_sized(23, 4000)
    sc = srp.Scene(mesh)
    dirs = synth.random_dirs(2300, 24)

    def batch(k0, n, B):
        return [(sc, np.full(mesh.n_dof, 0.05 * (k % 5) - 0.1), srp.params(dirs[k], n, B)) for k in range(k0, k0 + 8)]

    fa, fb, ga = batch(0, 160, 2), batch(8, 96, 1), batch(16, 128, 2)
    ref_a = srp.results_to_numpy(srp.eval_batch(fa)).copy()
    ref_b = srp.results_to_numpy(srp.eval_batch(fb)).copy()
    r, g = srp.eval_grad_batch(ga)
    ref_g, ref_gr = srp.results_to_numpy(r).copy(), g.cpu().numpy().copy()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = []
    for rep in range(3):
        oa = torch.empty(len(fa) * srp.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        ob = torch.empty_like(oa)
        og = torch.empty_like(oa)
        gg = torch.zeros_like(g)
        torch.cuda.synchronize()
        srp.eval_batch(fa, oa, streams[0])
        srp.eval_batch(fb, ob, streams[1])
        srp.eval_grad_batch(ga, og, gg, streams[2])
        outs.append((oa, ob, og, gg))
    torch.cuda.synchronize()
    for oa, ob, og, gg in outs:
        assert srp.results_to_numpy(oa).tobytes() == ref_a.tobytes()
        assert srp.results_to_numpy(ob).tobytes() == ref_b.tobytes()
        assert srp.results_to_numpy(og).tobytes() == ref_g.tobytes()
        assert gg.cpu().numpy().tobytes() == ref_gr.tobytes()


@pytest.mark.parametrize("n", [1, 2, 17, 100, 257, 600, 1030])
def test_ragged_and_tiny_grids(srp, n):
    """Grid sizes that are not multiples of the 16-pixel tile, down to one ray;
    600 and 1030 also split the reduction's first stage into 5 and 16 ranges."""
    mesh = synth.box_wing()
    sc = srp.Scene(mesh)
    sun = synth.random_dirs(2300 + n)[0]
    g = srp.eval(sc, sun, n, bounces=1, record=True)
    o = oracle.eval_srp(mesh, sun, n, bounces=1, record=True)
    rep = compare_eval(mesh, None, sun, n, 1, g, o)
    _show(f"ragged n={n}", rep)
    assert rep["primary_outside_band"] == 0 and rep["f_err_vis_matched"] <= F_TOL
    assert g["n_rays"] == n * n


def test_degenerate_cases(srp):
    """Edge-on plate (zero-area window): zero force, no hit.  A zero-area
    triangle is never hit.  Invalid parameters are errors."""
    plate = synth.plate((0, 0, 0), (1, 0, 0), (0, 1, 0))
    sc = srp.Scene(plate)
    g = srp.eval(sc, (1, 0, 0), 32, bounces=1)
    assert g["n_hits"] == 0 and not np.any(g["force"]) and not np.any(g["torque"])
    base = synth.plate((-1, -1, 0), (2, 0, 0), (0, 2, 0), rho=(0.3, 0.3))
    degen = np.array([[[-0.5, 0.0, 0.5], [0.5, 0.0, 0.5], [0.5, 0.0, 0.5]]])
    with_d = synth.merge_static(base, np.concatenate([base.verts[base.tris], degen]),
                                tri_mat=np.zeros(3, np.int32))
    a = srp.eval(srp.Scene(base), (0, 0, 1), 50, bounces=1)
    b = srp.eval(srp.Scene(with_d), (0, 0, 1), 50, bounces=1)
    assert np.array_equal(a["force"], b["force"]) and a["n_hits"] == b["n_hits"] == 2500
    for bad in (dict(n=0), dict(n=9000), dict(bounces=5), dict(sun_dir=(0, 0, 0)),
                dict(sun_dir=(np.nan, 0, 1))):
        kw = dict(sun_dir=(0, 0, 1), n=8, bounces=0)
        kw.update(bad)
        with pytest.raises(srp.SrpError):
            srp.eval(sc, kw["sun_dir"], kw["n"], bounces=kw["bounces"])
    with pytest.raises(srp.SrpError):
        srp.Scene(synth.box_wing()).set_angles([0.1])


@pytest.mark.parametrize("maker,n,B", [
    (lambda: synth.box_wing(), 96, 1),
    (lambda: synth.procedural_sized(23, 3000), 128, 2),
    (lambda: synth.box_wing_2axis(tess=6), 96, 2),
])
def test_adjoint_matches_finite_differences(srp, maker, n, B):
    """Hand-written adjoint (fixed visibility) against FP64 central finite
    differences (h = 1e-4) of the oracle's re-shade, every gradient block
    (rho_s, rho_d, theta, the photon-direction Jacobian) against its own
    largest entry: on the GPU's recorded hits (visibility matched) within
    G_TOL_VM, on the oracle's own recorded hits within G_TOL beyond the share
    of the rays whose hits differ."""
    mesh = maker()
    ang = np.linspace(-0.5, 0.7, mesh.n_dof)
    sc = srp.Scene(mesh)
    sc.set_angles(ang)
    for seed in (2401, 2402):
        sun = synth.random_dirs(seed)[0]
        g = srp.eval_grad(sc, sun, n, bounces=B, pressure=2.0)
        rec = srp.eval(sc, sun, n, bounces=B, pressure=2.0, record=True)
        assert np.array_equal(g["force"], rec["force"])
        o = oracle.eval_srp(mesh, sun, n, bounces=B, pressure=2.0, angles=ang, record=True)
        rep = grad_report(g, mesh, sun, n, B, o.grid, o.ids, rec["ids"], pressure=2.0, angles=ang,
                          dir_jacobian=True)
        print(f"adjoint {mesh.name} seed={seed} per-block err (oracle hits, GPU hits, flipped share): {rep}",
              flush=True)
        check_grads(rep)


def test_hinge_gradient_flat_plate_closed_form(srp):
    """A hinged plate lit along -z fills its window at every angle: the
    adjoint's hinge derivative is the derivative of the flat-plate law
    F(t) = P A cos t [(1-rs) d - 2 (rs cos t + rd/3) n(t)], cos t prefactor
    included (c' = -sin t, n' = y x n), and its coefficient terms are
    P A c (-d - 2 c n) and -(2/3) P A c n."""
    rs, rd, P, A = 0.35, 0.2, 1.9, 6.0
    sc = srp.Scene(synth.hinged_plate(2.0, 3.0, rho=(rs, rd)))
    d = np.array([0.0, 0.0, -1.0])
    for t in (0.45, -0.8, 1.1):
        sc.set_angles([t])
        g = srp.eval_grad(sc, (0, 0, 1), 32, bounces=1, pressure=P)
        n = np.array([np.sin(t), 0.0, np.cos(t)])
        c, cp = np.cos(t), -np.sin(t)
        npr = np.array([np.cos(t), 0.0, -np.sin(t)])
        law = (1 - rs) * d - 2 * (rs * c + rd / 3) * n
        dF = P * A * (cp * law - 2 * c * (rs * cp * n + (rs * c + rd / 3) * npr))
        print(f"hinged plate t={t}: adjoint {g['theta'][0]} closed form {dF}", flush=True)
        assert block_err(g["theta"][0], dF) <= 2e-6
        assert block_err(g["rho_s"][0], P * A * c * (-d - 2 * c * n)) <= 2e-6
        assert block_err(g["rho_d"][0], -2 / 3 * P * A * c * n) <= 2e-6


def test_uneven_batch_small(srp):
    """Uneven batch (scenes of 1k..20k triangles, grids 64..320, random
    angles, 1 bounce) in one launch; every item's batch result bitwise equal
    to its single recorded evaluation, which is compared with the oracle by
    the edge-band policy (ids outside the band equal, visibility-matched force
    and torque within F_TOL, plain force within what flipped rays carry)."""
    specs = synth.uneven_batch_specs(seed=4, n=8)
    entries, meshes = [], []
    for k, s in enumerate(specs):
        m = synth.procedural_sized(s["seed"], min(s["target_tris"], 20000))
        ang = np.zeros(m.n_dof)
        ang[0], ang[m.n_dof // 2] = s["root_angles"]
        n = max(64, s["n"] // 6)
        entries.append((srp.Scene(m), ang, srp.params(s["sun_dir"], n, 1)))
        meshes.append((m, ang, s["sun_dir"], n))
    out = srp.results_to_numpy(srp.eval_batch(entries))
    for k, (m, ang, sun, n) in enumerate(meshes):
        sc = entries[k][0]
        sc.set_angles(ang)
        single = srp.eval(sc, sun, n, bounces=1, record=True)
        assert np.array_equal(single["force"], out[k]["force"]), k
        assert np.array_equal(single["torque"], out[k]["torque"]), k
        o = oracle.eval_srp(m, sun, n, bounces=1, angles=ang, record=True)
        rep = compare_eval(m, ang, sun, n, 1, single, o)
        _show(f"uneven item {k}: T={m.n_tris} n={n}", rep)
        _check(rep)


def test_autograd_function(srp):
    """torch.autograd.Function over the batched adjoint: backward of a scalar
    loss equals the hand contraction of srp_eval_grad's Jacobians, and the
    coefficient gradient matches the oracle's finite differences."""
    import torch
    from paper_2608_07307_amd.autograd import srp_forces
    mesh = synth.procedural_sized(41, 2500)
    sc = srp.Scene(mesh)
    dirs = synth.fibonacci_dirs(5)
    rs = torch.tensor(mesh.mats[:, 0], dtype=torch.float64, device="cuda", requires_grad=True)
    rd = torch.tensor(mesh.mats[:, 1], dtype=torch.float64, device="cuda", requires_grad=True)
    th = torch.tensor(np.linspace(-0.4, 0.5, mesh.n_dof), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    F = srp_forces(rs, rd, th, sc, dirs, 96, bounces=1, pressure=3.0)
    w = torch.tensor(np.random.default_rng(0).normal(size=(5, 3)), dtype=torch.float64, device="cuda")
    (F * w).sum().backward()
    gs = np.zeros(mesh.n_mats); gd = np.zeros(mesh.n_mats); gt = np.zeros(mesh.n_dof)
    sc.set_angles(th.detach().cpu().numpy())
    for k in range(5):
        g = srp.eval_grad(sc, dirs[k], 96, bounces=1, pressure=3.0)
        assert np.array_equal(g["force"], F[k].detach().cpu().numpy())
        wk = w[k].cpu().numpy()
        gs += g["rho_s"] @ wk
        gd += g["rho_d"] @ wk
        gt += g["theta"] @ wk
    np.testing.assert_allclose(rs.grad.cpu().numpy(), gs, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(rd.grad.cpu().numpy(), gd, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(th.grad.cpu().numpy(), gt, rtol=1e-12, atol=1e-15)


def test_schedules_plans_and_autotune(srp):
    """Forces are bitwise identical under every schedule (per-patch partial
    sums), and so are gradients (per fixed patch group of each evaluation),
    which also equal each item's gradients in a batch of its own; a captured plan
    replays bitwise the direct batch, also after an update with new Sun
    directions and angles; the autotuner returns a valid schedule that is
    then used."""
    import torch
    mesh = synth.procedural_sized(51, 5000)
    sc = srp.Scene(mesh)
    dirs = synth.fibonacci_dirs(24)
    rng = np.random.default_rng(51)
    angs = rng.uniform(-1.0, 1.0, size=(24, mesh.n_dof))
    entries = [(sc, angs[k % 6], srp.params(dirs[k], [64, 96, 160][k % 3], k % 3)) for k in range(24)]
    ref = srp.results_to_numpy(srp.eval_batch(entries)).copy()
    for ppc, bpc in ((1, 1), (2, 3), (3, 2), (8, 0), (16, 2), (64, 4), (0, 0)):
        srp.set_schedule(ppc, bpc)
        got = srp.results_to_numpy(srp.eval_batch(entries))
        assert got.tobytes() == ref.tobytes(), (ppc, bpc)
    # gradients: the adjoint's chunks are fixed patch groups of each evaluation,
    # so the gradient bits do not depend on the schedule either, and a batch
    # item's gradients are bitwise its single evaluation's
    gref = None
    for ppc, bpc in ((1, 1), (8, 0), (64, 4), (0, 0), (2, 3)):
        srp.set_schedule(ppc, bpc)
        gres, grad = srp.eval_grad_batch(entries)
        g = grad.cpu().numpy()
        assert srp.results_to_numpy(gres)["force"].tobytes() == ref["force"].tobytes()
        if gref is None:
            gref = g.copy()
        assert g.tobytes() == gref.tobytes(), (ppc, bpc)
    srp.set_schedule(0, 0)
    for k in (0, 7, 23):
        _, g1 = srp.eval_grad_batch([entries[k]])
        assert g1.cpu().numpy()[0].tobytes() == gref[k].tobytes(), k
    plan = srp.Plan(entries)
    for _ in range(3):
        out = srp.results_to_numpy(plan.launch())
        torch.cuda.synchronize()
        assert out.tobytes() == ref.tobytes()
    dirs2 = synth.fibonacci_dirs(48)[24:]
    entries2 = [(sc, angs[(k + 1) % 6], srp.params(dirs2[k], [64, 96, 160][k % 3], k % 3)) for k in range(24)]
    plan.update(entries2)
    out2 = srp.results_to_numpy(plan.launch())
    ref2 = srp.results_to_numpy(srp.eval_batch(entries2))
    assert out2.tobytes() == ref2.tobytes()
    r, b, ms = srp.autotune(entries)
    print(f"autotune: patches/chunk {r} blocks/CU {b} {ms:.3f} ms", flush=True)
    assert r in (1, 2, 4, 8, 16, 32, 64) and b >= 1 and ms > 0
    assert srp.results_to_numpy(srp.eval_batch(entries)).tobytes() == ref.tobytes()
    # the autotuner of the forward + adjoint launch (its own gradient buffer), then
    # a gradient batch under the tuned schedule
    rg, bg, msg = srp.autotune(entries, grad=True)
    print(f"autotune (adjoint): patches/chunk {rg} blocks/CU {bg} {msg:.3f} ms", flush=True)
    assert rg in (1, 2, 4, 8, 16, 32, 64) and bg >= 1 and msg > 0
    res, grad = srp.eval_grad_batch(entries)
    assert srp.results_to_numpy(res)["force"].tobytes() == ref["force"].tobytes()
    assert np.isfinite(grad.cpu().numpy()).all()
    plan.close()


def test_direction_jacobian_plate_closed_form(srp):
    """A plate that fills its window: dF/dd = P A [-L n^T + c ((1-rs) I +
    2 rs n n^T)], L = (1-rs) d - 2 (rs c + rd/3) n, c = -n.d (by hand)."""
    rs, rd, P = 0.35, 0.25, 1.7
    sun = np.array([0.3, -0.2, 1.0])
    d = -sun / np.linalg.norm(sun)
    h = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    u = np.cross(h, d)
    u /= np.linalg.norm(u)
    v = np.cross(d, u)
    ev = 1.5 * (np.cos(0.6) * v + np.sin(0.6) * d)
    mesh = synth.plate(origin=0.3 * u - 0.7 * v + 0.2 * d, eu=2.0 * u, ev=ev, rho=(rs, rd))
    sc = srp.Scene(mesh)
    g = srp.eval_grad(sc, sun, 32, bounces=1, pressure=P)
    n = np.cross(u, ev)
    n /= np.linalg.norm(n)
    if n @ d > 0:
        n = -n
    c = -n @ d
    L = (1 - rs) * d - 2 * (rs * c + rd / 3) * n
    J = P * 3.0 * (-np.outer(L, n) + c * ((1 - rs) * np.eye(3) + 2 * rs * np.outer(n, n)))
    np.testing.assert_allclose(g["dir"], J, rtol=2e-5, atol=2e-5 * np.abs(J).max())


def test_autograd_sun_direction_and_attitude(srp):
    """Sun-direction gradients through the autograd Function: the backward of
    a loss equals the hand contraction of dF/dd with dd/ds; an attitude R(w)
    composed in torch (F_inertial = R F(R^T s)) has a w-gradient that matches
    central differences of the oracle's frozen re-shade at the rotated
    direction."""
    import torch
    from paper_2608_07307_amd.autograd import srp_forces
    mesh = synth.procedural_sized(42, 2500)
    sc = srp.Scene(mesh)
    th0 = np.linspace(-0.3, 0.4, mesh.n_dof)
    rs = torch.tensor(mesh.mats[:, 0], dtype=torch.float64, device="cuda")
    rd = torch.tensor(mesh.mats[:, 1], dtype=torch.float64, device="cuda")
    th = torch.tensor(th0, dtype=torch.float64, device="cuda")
    dirs = torch.tensor(synth.fibonacci_dirs(4) * 2.0, dtype=torch.float64, device="cuda", requires_grad=True)
    F = srp_forces(rs, rd, th, sc, dirs, 96, bounces=1, pressure=3.0)
    w = torch.tensor(np.random.default_rng(1).normal(size=(4, 3)), dtype=torch.float64, device="cuda")
    (F * w).sum().backward()
    sc.set_angles(th0)
    for k in range(4):
        s = dirs[k].detach().cpu().numpy()
        g = srp.eval_grad(sc, s, 96, bounces=1, pressure=3.0)
        sh = s / np.linalg.norm(s)
        dds = -(np.eye(3) - np.outer(sh, sh)) / np.linalg.norm(s)
        np.testing.assert_allclose(dirs.grad[k].cpu().numpy(), w[k].cpu().numpy() @ g["dir"] @ dds,
                                   rtol=1e-12, atol=1e-15)
    # attitude: body frame = R(omega)^T inertial; F_inertial = R F_body(R^T s)
    s_in = np.array([0.4, -0.7, 0.6])

    def rot(om):
        th_ = torch.linalg.norm(om)
        K = torch.zeros(3, 3, dtype=om.dtype, device=om.device)
        K[0, 1], K[0, 2], K[1, 0], K[1, 2], K[2, 0], K[2, 1] = -om[2], om[1], om[2], -om[0], -om[1], om[0]
        return torch.eye(3, dtype=om.dtype, device=om.device) + torch.sin(th_) / th_ * K + \
            (1 - torch.cos(th_)) / th_ ** 2 * K @ K

    om = torch.tensor([0.2, -0.1, 0.3], dtype=torch.float64, device="cuda", requires_grad=True)
    R = rot(om)
    s_body = (R.T @ torch.tensor(s_in, dtype=torch.float64, device="cuda")).reshape(1, 3)
    Fb = srp_forces(rs, rd, th, sc, s_body, 96, bounces=1, pressure=3.0)
    wi = torch.tensor([0.3, 1.0, -0.5], dtype=torch.float64, device="cuda")
    ((R @ Fb[0]) * wi).sum().backward()
    sb = s_body.detach().cpu().numpy()[0]
    o = oracle.eval_srp(mesh, sb, 96, bounces=1, pressure=3.0, angles=th0, record=True)

    def loss(om_np):
        Rn = rot(torch.tensor(om_np, dtype=torch.float64)).numpy()
        d_body = Rn.T @ (-s_in / np.linalg.norm(s_in))
        Fbn = oracle.shade_frozen_dir(mesh, 96, 1, o.grid, o.ids, d_body, pressure=3.0, angles=th0)
        return (Rn @ Fbn) @ wi.cpu().numpy()

    hh = 1e-6
    fd = np.array([(loss(om.detach().cpu().numpy() + hh * e) - loss(om.detach().cpu().numpy() - hh * e)) / (2 * hh)
                   for e in np.eye(3)])
    err = np.abs(om.grad.cpu().numpy() - fd).max() / np.abs(fd).max()
    print(f"attitude gradient: autograd {om.grad.cpu().numpy()}, oracle FD {fd}, rel err {err:.2e}", flush=True)
    assert err <= 2e-4


def test_profile_hooks_time_trace_and_whole_launch(srp):
    """The measurement hooks: while profiling is on, every batch launch adds one
    trace-kernel interval and one whole-launch interval (staging upload through
    result copy), the whole launch lasting at least as long as its trace kernel;
    once it is off, nothing more is recorded."""
    m = synth.box_wing()
    sc = srp.Scene(m)
    entries = [(sc, np.zeros(m.n_dof), srp.params(synth.random_dirs(3100 + k)[0], 96, 1)) for k in range(8)]
    srp.eval_batch(entries)
    srp.profile(True)
    for _ in range(3):
        srp.eval_batch(entries)
    ms_t, n_t = srp.profile_read()
    ms_l, n_l = srp.profile_read_launch()
    srp.profile(False)
    assert n_t == 3 and n_l == 3
    assert 0.0 < ms_t <= ms_l
    srp.eval_batch(entries)
    assert srp.profile_read() == (0.0, 0)
    assert srp.profile_read_launch() == (0.0, 0)
