"""CPU check of the library's ray traversal (csrc/trace.h), built with the
host compiler under AddressSanitizer and UndefinedBehaviorSanitizer
(tests/host_trace/trace_check.cpp; the scene and its articulation slot come
from the library's own host builder, csrc/scene.cpp).

The per-lane LDS ring is shrunk from 16 entries to 2, so nearly every ray
runs the spill path, and the ring and spill arrays are exactly their sizes,
so a stack access out of range (an LDS ring slot past its end, a spill entry
past its area) stops the run with a sanitizer report.  Checked: primary hit
ids against the FP64 oracle (edge band excepted) on random scenes, secondary
rays with an excluded triangle and t > tmin, empty-stack pops (every ray ends
by popping the last entry), every ray's deepest stack within the builder's
worst-case bound, and overflow reported (not written past the spill area)
when the traversal is built with a stack shallower than the hierarchy needs.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from parity import classify_primary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_07307_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host_trace", "trace_check.cpp")
HIP_INC = "/opt/rocm/include"

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INC),
                                reason="needs g++ and the HIP headers")

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
COMMON = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", HIP_INC, "-I", os.path.join(ROOT, "include"),
          "-I", CSRC]


@pytest.fixture(scope="module")
def build(tmp_path_factory):
    """Builds the harness: the scene builder at the library's own stack depth,
    the traversal with a 2-entry ring and the given depth (None = the
    library's)."""
    tmp = tmp_path_factory.mktemp("trace_host")
    scene_o = tmp / "scene.o"
    subprocess.run(["g++", *COMMON, *SAN, "-c", os.path.join(CSRC, "scene.cpp"), "-o", str(scene_o)], check=True)
    cache = {}

    def make(depth=None):
        if depth in cache:
            return cache[depth]
        exe = tmp / f"trace_check_{depth or 'lib'}"
        flags = ["-DSRP_STACK_LDS=2"] + ([f"-DSRP_STACK_DEPTH={depth}"] if depth else [])
        subprocess.run(["g++", *COMMON, *SAN, *flags, HARNESS, str(scene_o), "-o", str(exe)], check=True)
        cache[depth] = exe
        return exe

    return make, tmp


def _run(exe, tmp, mesh, angles, rays, skip=None, planar_out=None):
    """rays: (k, 8) float64 rows o(3), d(3), tmin, exclude; skip: per ray the
    instance skipped whole (default none).  planar_out (a list) receives the
    builder's per-node planarity flags."""
    from paper_2608_07307_amd import _mesh_arrays
    verts, tris, tm, tn, mats, nodes = _mesh_arrays(mesh)
    ang = np.zeros(mesh.n_dof) if angles is None else np.asarray(angles, np.float64)
    rec = np.zeros(len(rays), dtype=[("o", "<f4", 3), ("d", "<f4", 3), ("tmin", "<f4"), ("ex", "<i4"),
                                     ("sk", "<i4")])
    rec["o"], rec["d"], rec["tmin"], rec["ex"] = rays[:, :3], rays[:, 3:6], rays[:, 6], rays[:, 7]
    rec["sk"] = -1 if skip is None else skip
    inp, out = tmp / "in.bin", tmp / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([verts.shape[0], tris.shape[0]], "<i8").tobytes())
        f.write(np.array([len(mesh.mats), len(mesh.parent), mesh.n_dof, len(rays)], "<i4").tobytes())
        for a in (verts, tris, tm, tn):
            f.write(a.tobytes())
        f.write(bytes(mats))
        f.write(bytes(nodes))
        f.write(np.ascontiguousarray(ang, "<f8").tobytes())
        f.write(rec.tobytes())
    r = subprocess.run([str(exe), str(inp), str(out)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0"))
    assert r.returncode == 0, r.stderr[-3000:]
    raw = open(out, "rb").read()
    status, worst, nn = np.frombuffer(raw[:12], "<i4")
    if planar_out is not None:
        planar_out.extend(int(x) for x in np.frombuffer(raw[12:12 + 4 * nn], "<i4"))
    res = np.frombuffer(raw[12 + 4 * nn:], dtype=[("ok", "<i4"), ("id", "<i4"), ("t", "<f4"), ("nbox", "<u4"),
                                        ("ntri", "<u4"), ("deep", "<i4")])
    return int(status), int(worst), res


def _primary_rays(grid, n):
    """The oracle's pixel-centre rays (FP64 origins rounded to FP32)."""
    j, i = np.divmod(np.arange(n * n), n)
    a = grid["umin"] + (i + 0.5) * grid["wu"] / n
    b = grid["vmin"] + (j + 0.5) * grid["wv"] / n
    o = a[:, None] * grid["u"] + b[:, None] * grid["v"] + grid["h0"] * grid["d"]
    return np.concatenate([o, np.tile(grid["d"], (n * n, 1)), np.zeros((n * n, 1)), -np.ones((n * n, 1))], 1)


@pytest.mark.parametrize("maker,seed", [
    (lambda: synth.box_wing(), 1),
    (lambda: synth.procedural_sized(61, 3000), 2),
    (lambda: synth.box_wing_2axis(tess=6), 3),
    (lambda: synth.procedural_sized(62, 20000), 4),
])
def test_primary_ids_against_oracle(build, maker, seed):
    make, tmp = build
    mesh = maker()
    rng = np.random.default_rng(seed)
    ang = rng.uniform(-1.0, 1.0, mesh.n_dof)
    sun = synth.random_dirs(7000 + seed)[0]
    n = 48
    o = oracle.eval_srp(mesh, sun, n, bounces=0, angles=ang, record=True)
    status, worst, res = _run(make(), tmp, mesh, ang, _primary_rays(o.grid, n))
    assert status == 0 and (res["ok"] == 1).all()
    assert (res["deep"] <= worst).all(), (res["deep"].max(), worst)
    if mesh.n_tris > 1000:
        assert res["deep"].max() > 2      # the 2-entry ring overflowed into the spill area
    m, outside, frac = classify_primary(mesh, ang, o.grid, n, o.ids[:, 0], res["id"])
    print(f"{mesh.name}: {m} ids differ ({frac:.2e} of rays in the edge band), deepest stack "
          f"{res['deep'].max()} of the bound {worst}", flush=True)
    assert outside == 0
    hit = res["id"] >= 0
    np.testing.assert_allclose(res["t"][hit], o.ts[hit, 0], rtol=1e-4, atol=1e-4 * o.grid["L"])


def test_secondary_rays_exclude_and_tmin(build):
    """Rays leaving a hit along its specular direction, with the hit triangle
    excluded and t > 1e-6 L: the first hit equals the oracle's recorded
    secondary hit outside the edge band of that ray."""
    make, tmp = build
    mesh = synth.procedural_sized(63, 5000)
    ang = np.linspace(-0.6, 0.6, mesh.n_dof)
    sun = synth.random_dirs(7100)[0]
    n = 48
    o = oracle.eval_srp(mesh, sun, n, bounces=1, angles=ang, record=True)
    sec = np.nonzero(o.ids[:, 1] >= 0)[0]
    assert sec.size > 20
    world = oracle.articulate(mesh, ang)
    prim = _primary_rays(o.grid, n)[sec]
    d = o.grid["d"]
    x = prim[:, :3] + o.ts[sec, 0][:, None] * d
    W = world[o.ids[sec, 0]]
    nrm = np.cross(W[:, 1] - W[:, 0], W[:, 2] - W[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    nrm *= -np.sign(nrm @ d)[:, None]
    r = d + 2 * (-(nrm @ d))[:, None] * nrm
    rays = np.concatenate([x, r, np.full((len(sec), 1), 1e-6 * o.grid["L"]), o.ids[sec, 0][:, None]], 1)
    status, worst, res = _run(make(), tmp, mesh, ang, rays)
    assert status == 0 and (res["ok"] == 1).all() and (res["deep"] <= worst).all()
    same = (res["id"] == o.ids[sec, 1]).mean()
    print(f"secondary rays: {same:.4f} of {len(sec)} agree with the oracle", flush=True)
    assert same > 0.99
    assert not np.any(res["id"] == o.ids[sec, 0])      # the source triangle is never hit again


def _planar_nodes(mesh):
    """Nodes whose triangles all lie within 1e-9 x the mesh's coordinate scale
    of the plane through the node's first vertex with its summed normal
    (numpy, independent of the library's builder)."""
    from paper_2608_07307_amd import _mesh_arrays
    verts, tris, _, tn, _, _ = _mesh_arrays(mesh)
    V, T = verts.reshape(-1, 3), tris.reshape(-1, 3)
    scale = np.abs(V[T.ravel()]).max()
    out = []
    for k in range(len(mesh.parent)):
        P = V[T[tn == k]]
        if not len(P):
            out.append(0)
            continue
        nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]).sum(0)
        nrm /= np.linalg.norm(nrm)
        out.append(int(np.abs((P.reshape(-1, 3) - P[0, 0]) @ nrm).max() <= 1e-9 * scale))
    return out, np.asarray(tn)


def test_secondary_rays_skip_the_planar_instance_they_leave(build):
    """A ray leaving a triangle of a node whose triangles lie in one plane
    cannot meet that node again, so the traversal may skip it whole.  The
    builder flags exactly the planar nodes (the panel segments here, not the
    bus or the dish), and first-bounce rays traced with their source node
    skipped meet the same triangles at the same distances as without the
    skip, with fewer box tests; the only rays allowed to differ are those
    whose unskipped hit lies in the node they leave (an FP32 re-hit of the
    plane next to a grazing origin), and there must be none at this size."""
    make, tmp = build
    mesh = synth.procedural_sized(64, 6000)
    ang = np.linspace(-0.9, 0.7, mesh.n_dof)
    n = 64
    expect, node_of = _planar_nodes(mesh)
    assert 0 < sum(expect) < len(expect)
    nsec = 0
    for seed in (7200, 7201, 7202):
        sun = synth.random_dirs(seed)[0]
        o = oracle.eval_srp(mesh, sun, n, bounces=1, angles=ang, record=True)
        src = np.nonzero(o.ids[:, 0] >= 0)[0]
        world = oracle.articulate(mesh, ang)
        d = o.grid["d"]
        x = _primary_rays(o.grid, n)[src, :3] + o.ts[src, 0][:, None] * d
        W = world[o.ids[src, 0]]
        nrm = np.cross(W[:, 1] - W[:, 0], W[:, 2] - W[:, 0])
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        nrm *= -np.sign(nrm @ d)[:, None]
        r = d + 2 * (-(nrm @ d))[:, None] * nrm
        rays = np.concatenate([x, r, np.full((len(src), 1), 1e-6 * o.grid["L"]), o.ids[src, 0][:, None]], 1)
        planar = []
        status, worst, r0 = _run(make(), tmp, mesh, ang, rays, planar_out=planar)
        assert status == 0 and planar == expect
        leave = node_of[o.ids[src, 0]]
        skip = np.where(np.asarray(planar)[leave] == 1, leave, -1).astype(np.int32)
        status, worst, r1 = _run(make(), tmp, mesh, ang, rays, skip=skip)
        assert status == 0 and (r0["ok"] == 1).all() and (r1["ok"] == 1).all()
        rehit = (skip >= 0) & (r0["id"] >= 0) & (node_of[np.maximum(r0["id"], 0)] == skip)
        assert not rehit.any()
        assert np.array_equal(r1["id"], r0["id"]) and np.array_equal(r1["t"], r0["t"])
        assert (skip >= 0).mean() > 0.3
        assert r1["nbox"].sum() < 0.9 * r0["nbox"].sum()
        nsec += len(src)
        print(f"sun {seed}: {len(src)} rays, {(skip >= 0).mean():.2f} leave a planar node; box tests per ray "
              f"{r0['nbox'].mean():.1f} -> {r1['nbox'].mean():.1f}", flush=True)
    assert nsec > 1000


def test_deep_hierarchy_and_overflow(build):
    """4,096 stacked plates seen face-on: every child box on the way to the
    top plate is hit, so the descent pushes three entries per 4-wide level.
    At the library's depth every ray reaches the top plate within the
    builder's bound; with the traversal built for 6 entries every ray reports
    the overflow (and nothing is written past the spill area)."""
    make, tmp = build
    mesh = synth.stacked_plates(1 << 12)
    n = 8
    grid = oracle.grid_of(mesh, (0, 0, 1), n)
    rays = _primary_rays(grid, n)
    status, worst, res = _run(make(), tmp, mesh, None, rays)
    top = (1 << 12) - 1
    assert status == 0 and (res["ok"] == 1).all() and (res["id"] // 2 == top).all()
    assert 6 < res["deep"].max() <= worst
    status, worst6, res6 = _run(make(6), tmp, mesh, None, rays)
    assert status == 0 and worst6 == worst and (res6["ok"] == 0).all()
