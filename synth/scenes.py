"""Seeded procedural spacecraft meshes (geometry + kinematic tree + materials).

The paper's own meshes (a 39,257-triangle Parker Solar Probe model and a
212-triangle box-wing satellite, Sec. 5.1 table of spacecraft models) are not
available, so every workload here is a seeded procedural stand-in with the
same structure: a bus, optical parts with per-part absorbed/specular/diffuse
coefficients, and solar arrays attached through a rooted kinematic tree whose
edges carry a pivot, rotation axes and angular intervals (Sec. 4.4.1).

Conventions shared by every consumer (oracle and library alike):
  * units are metres; vertices are in the rest-pose body frame;
  * node 0 is the root (parent -1, no degrees of freedom) and parent[k] < k,
    so node order is a topological order of the tree;
  * a node's degrees of freedom follow node order, then axis order, in the
    flat hinge-angle vector (n_dof = sum of n_axes);
  * a triangle's corners are moved by the transform of the triangle's node;
    generators never share a vertex between nodes;
  * materials hold (rho_s, rho_d); rho_a = 1 - rho_s - rho_d.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Scene:
    verts: np.ndarray      # (V,3) float64
    tris: np.ndarray       # (T,3) int32
    tri_mat: np.ndarray    # (T,)  int32
    tri_node: np.ndarray   # (T,)  int32
    mats: np.ndarray       # (M,2) float64: rho_s, rho_d
    parent: np.ndarray     # (K,)  int32
    is_panel: np.ndarray   # (K,)  int32
    pivot: np.ndarray      # (K,3) float64
    n_axes: np.ndarray     # (K,)  int32
    axes: np.ndarray       # (K,3,3) float64, rows = axes (unused rows zero)
    lo: np.ndarray         # (K,3) float64, radians
    hi: np.ndarray         # (K,3) float64, radians
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_mats(self) -> int:
        return int(self.mats.shape[0])

    @property
    def n_dof(self) -> int:
        return int(self.n_axes.sum())

    def zero_angles(self) -> np.ndarray:
        return np.zeros(self.n_dof, dtype=np.float64)

    def with_mats(self, mats) -> "Scene":
        m = np.ascontiguousarray(np.asarray(mats, dtype=np.float64).reshape(-1, 2))
        return Scene(self.verts, self.tris, self.tri_mat, self.tri_node, m,
                     self.parent, self.is_panel, self.pivot, self.n_axes,
                     self.axes, self.lo, self.hi, self.name, dict(self.meta))


class _Builder:
    """Accumulates mesh parts and tree nodes; emits a Scene."""

    def __init__(self):
        self.v, self.t, self.m, self.n = [], [], [], []
        self.nv = 0
        self.nodes = []  # (parent, is_panel, pivot, axes list, lo list, hi list)

    def node(self, parent=-1, is_panel=0, pivot=(0, 0, 0), axes=(), lo=(), hi=()):
        self.nodes.append((parent, is_panel, pivot, list(axes), list(lo), list(hi)))
        return len(self.nodes) - 1

    def tris(self, verts, tris, node, mats):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self.v.append(verts)
        self.t.append(tris + self.nv)
        self.nv += verts.shape[0]
        mats = np.broadcast_to(np.asarray(mats, dtype=np.int64), (tris.shape[0],))
        self.m.append(np.array(mats))
        self.n.append(np.full(tris.shape[0], node, dtype=np.int64))

    def quad_grid(self, origin, eu, ev, nu, nv, node, mat_fn):
        """nu x nv quads spanning origin + [0,1]eu + [0,1]ev, 2 tris per quad."""
        o, eu, ev = (np.asarray(x, dtype=np.float64) for x in (origin, eu, ev))
        a = np.arange(nu + 1)[:, None] / nu
        b = np.arange(nv + 1)[None, :] / nv
        verts = o + a[..., None] * eu + b[..., None] * ev          # (nu+1, nv+1, 3)
        idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
        p00, p10 = idx[:-1, :-1], idx[1:, :-1]
        p11, p01 = idx[1:, 1:], idx[:-1, 1:]
        t1 = np.stack([p00, p10, p11], -1).reshape(-1, 3)
        t2 = np.stack([p00, p11, p01], -1).reshape(-1, 3)
        tris = np.stack([t1, t2], 1).reshape(-1, 3)
        ai, bi = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
        qm = np.asarray(mat_fn(ai.reshape(-1), bi.reshape(-1)), dtype=np.int64)
        self.tris(verts.reshape(-1, 3), tris, node, np.repeat(np.broadcast_to(qm, (nu * nv,)), 2))

    def box(self, center, half, node, mat):
        c, h = np.asarray(center, float), np.asarray(half, float)
        s = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], float)
        verts = c + s * h
        # corner index = 4*ix + 2*iy + iz (ix,iy,iz in {0,1})
        faces = [(0, 1, 3, 2), (4, 6, 7, 5),   # x = -h, x = +h
                 (0, 4, 5, 1), (2, 3, 7, 6),   # y = -h, y = +h
                 (0, 2, 6, 4), (1, 5, 7, 3)]   # z = -h, z = +h
        tris = []
        for a, b, cc, d in faces:
            tris += [(a, b, cc), (a, cc, d)]
        self.tris(verts, tris, node, mat)

    def dish(self, center, apex_z, radius, focal, rings, sectors, node, mat):
        """Single-layer paraboloid z = apex_z + r^2/(4 focal) on an (r, phi) grid.

        Ring 0 sits at r = 0 with `sectors` coincident vertices, so the first
        ring carries `sectors` zero-area triangles (a deliberate degenerate case).
        """
        r = radius * np.arange(rings + 1) / rings
        phi = 2 * np.pi * np.arange(sectors) / sectors
        R, P = np.meshgrid(r, phi, indexing="ij")
        verts = np.stack([center[0] + R * np.cos(P), center[1] + R * np.sin(P),
                          apex_z + R * R / (4 * focal)], -1).reshape(-1, 3)
        idx = np.arange((rings + 1) * sectors).reshape(rings + 1, sectors)
        jn = np.roll(np.arange(sectors), -1)
        p00, p10 = idx[:-1, :], idx[1:, :]
        p11, p01 = idx[1:, jn], idx[:-1, jn]
        t1 = np.stack([p00, p10, p11], -1).reshape(-1, 3)
        t2 = np.stack([p00, p11, p01], -1).reshape(-1, 3)
        tris = np.stack([t1, t2], 1).reshape(-1, 3)
        self.tris(verts, tris, node, mat)

    def build(self, mats, name="", meta=None) -> Scene:
        K = len(self.nodes)
        parent = np.array([n[0] for n in self.nodes], np.int32)
        is_panel = np.array([n[1] for n in self.nodes], np.int32)
        pivot = np.array([n[2] for n in self.nodes], np.float64).reshape(K, 3)
        n_axes = np.array([len(n[3]) for n in self.nodes], np.int32)
        axes = np.zeros((K, 3, 3))
        lo = np.zeros((K, 3))
        hi = np.zeros((K, 3))
        for k, n in enumerate(self.nodes):
            for a, (ax, l, h) in enumerate(zip(n[3], n[4], n[5])):
                ax = np.asarray(ax, float)
                axes[k, a] = ax / np.linalg.norm(ax)
                lo[k, a], hi[k, a] = l, h
        return Scene(
            verts=np.ascontiguousarray(np.concatenate(self.v)),
            tris=np.ascontiguousarray(np.concatenate(self.t).astype(np.int32)),
            tri_mat=np.ascontiguousarray(np.concatenate(self.m).astype(np.int32)),
            tri_node=np.ascontiguousarray(np.concatenate(self.n).astype(np.int32)),
            mats=np.ascontiguousarray(np.asarray(mats, np.float64).reshape(-1, 2)),
            parent=parent, is_panel=is_panel, pivot=pivot, n_axes=n_axes,
            axes=axes, lo=lo, hi=hi, name=name, meta=dict(meta or {}),
        )


def _random_mats(rng, n, hi=0.6, cap=0.9):
    """rho_s, rho_d ~ U(0, hi) each, rejected until rho_s + rho_d <= cap."""
    out = []
    while len(out) < n:
        s, d = rng.uniform(0.0, hi, size=2)
        if s + d <= cap:
            out.append((s, d))
    return np.array(out)


HALF_PI = np.pi / 2


# --------------------------------------------------------------------------
# small test meshes
# --------------------------------------------------------------------------
def plate(origin, eu, ev, rho=(0.3, 0.2), nu=1, nv=1) -> Scene:
    """Flat parallelogram origin + [0,1]eu + [0,1]ev, nu x nv quads, 1 material."""
    b = _Builder()
    root = b.node()
    b.quad_grid(origin, eu, ev, nu, nv, root, lambda a, c: 0 * a)
    return b.build([rho], name="plate")


def stacked_plates(n_plates=1 << 19, spacing=1e-5, size=1.0, rho=(0.4, 0.2), power=1.0) -> Scene:
    """n_plates identical size x size squares (2 triangles each) at heights
    z_i = spacing * i**power: a ray along -z passes through every plate, so
    both children of every hierarchy node on the way to the top plate are hit
    (a traversal stack as deep as the tree; power > 1 crowds the plates
    towards z = 0, which makes the tree deeper than a balanced one)."""
    n = int(n_plates)
    z = np.arange(n, dtype=np.float64) ** power * spacing
    sq = np.array([[0, 0], [size, 0], [size, size], [0, size]], np.float64)
    verts = np.empty((n, 4, 3))
    verts[:, :, :2] = sq[None]
    verts[:, :, 2] = z[:, None]
    base = 4 * np.arange(n, dtype=np.int64)[:, None]
    tris = np.concatenate([base + np.array([0, 1, 2]), base + np.array([0, 2, 3])], axis=1).reshape(-1, 3)
    one = np.zeros(1, np.int32)
    return Scene(verts.reshape(-1, 3), tris.astype(np.int32), np.zeros(2 * n, np.int32), np.zeros(2 * n, np.int32),
                 np.array([rho], np.float64), np.array([-1], np.int32), one, np.zeros((1, 3)), one,
                 np.zeros((1, 3, 3)), np.zeros((1, 3)), np.zeros((1, 3)), name="stacked_plates")


def hinged_plate(width=2.0, length=3.0, rho=(0.3, 0.2), axis=(0, 1, 0),
                 pivot=(0, 0, 0), lim=HALF_PI) -> Scene:
    """Root with no triangles + one panel node: plate x in [-w/2,w/2],
    y in [0,length], z = 0, rotating about `axis` through `pivot`."""
    b = _Builder()
    root = b.node()
    p = b.node(parent=root, is_panel=1, pivot=pivot, axes=[axis], lo=[-lim], hi=[lim])
    b.quad_grid((-width / 2, 0, 0), (width, 0, 0), (0, length, 0), 1, 1, p, lambda a, c: 0 * a)
    return b.build([rho], name="hinged_plate")


def cube(half=0.5, rho=(0.3, 0.2), center=(0, 0, 0)) -> Scene:
    b = _Builder()
    root = b.node()
    b.box(center, (half, half, half), root, 0)
    return b.build([rho], name="cube")


def dihedral(L=1.0, H=1.0, rho=(1.0, 0.0), rho_b=None) -> Scene:
    """Two L x H faces meeting at 90 deg along the x axis: face A in z=0
    (y in [0,H]), face B in y=0 (z in [0,H]); the corner opens towards +y+z.
    Face B takes material rho_b (material 1) when given, else face A's."""
    b = _Builder()
    root = b.node()
    b.quad_grid((0, 0, 0), (L, 0, 0), (0, H, 0), 1, 1, root, lambda a, c: 0 * a)
    mb = 0 if rho_b is None else 1
    b.quad_grid((0, 0, 0), (L, 0, 0), (0, 0, H), 1, 1, root, lambda a, c: 0 * a + mb)
    return b.build([rho] if rho_b is None else [rho, rho_b], name="dihedral")


def icosphere(R=1.0, subdiv=3, rho=(0.3, 0.2)) -> Scene:
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, float) / np.linalg.norm(p) for p in v]
    for _ in range(subdiv):
        cache, nf = {}, []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b_, c in f:
            ab, bc, ca = mid(a, b_), mid(b_, c), mid(c, a)
            nf += [(a, ab, ca), (b_, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    b = _Builder()
    root = b.node()
    b.tris(R * np.array(verts), f, root, 0)
    return b.build([rho], name=f"icosphere{subdiv}")


# --------------------------------------------------------------------------
# workload meshes
# --------------------------------------------------------------------------
def box_wing(rho_bus=(0.2, 0.4), rho_panel=(0.05, 0.1)) -> Scene:
    """Box-wing satellite: 1 m cube bus (12 tris) and two 2 x 5 m flat panels
    (2 tris each) on hinges about y through (0, +-1.5, 0), range +-90 deg,
    rest normal +z.  16 triangles, 3 nodes, 2 degrees of freedom."""
    b = _Builder()
    root = b.node()
    b.box((0, 0, 0), (0.5, 0.5, 0.5), root, 0)
    for s in (1.0, -1.0):
        p = b.node(parent=root, is_panel=1, pivot=(0, 1.5 * s, 0), axes=[(0, 1, 0)],
                   lo=[-HALF_PI], hi=[HALF_PI])
        y0 = 1.5 if s > 0 else -6.5
        b.quad_grid((-1, y0, 0), (2, 0, 0), (0, 5, 0), 1, 1, p, lambda a, c: 1 + 0 * a)
    return b.build([rho_bus, rho_panel], name="box_wing")


def box_wing_2axis(rho_bus=(0.2, 0.4), rho_panel=(0.05, 0.1), tess=1) -> Scene:
    """The box-wing with two-axis wings: each 2 x 5 m panel turns about its
    support axis (y, through (0, +-1.5, 0), +-90 deg), then folds about a hinge
    across the wing (x, through the same point, +-45 deg); axes composed in
    that order.  tess x tess quads per panel.  4 degrees of freedom."""
    b = _Builder()
    root = b.node()
    b.box((0, 0, 0), (0.5, 0.5, 0.5), root, 0)
    for s in (1.0, -1.0):
        p = b.node(parent=root, is_panel=1, pivot=(0, 1.5 * s, 0), axes=[(0, 1, 0), (1, 0, 0)],
                   lo=[-HALF_PI, -HALF_PI / 2], hi=[HALF_PI, HALF_PI / 2])
        y0 = 1.5 if s > 0 else -6.5
        b.quad_grid((-1, y0, 0), (2, 0, 0), (0, 5, 0), tess, tess, p, lambda a, c: 1 + 0 * a)
    return b.build([rho_bus, rho_panel], name="box_wing_2axis")


def _panel_chain(b, root, sign, axis_along, axis_across, root_dist, length, width,
                 n_segments, nx, ny, mat_fn, lim=HALF_PI):
    """A wing of `n_segments` rigid segments along +-axis_along.

    Segment 0 hangs off the root by a joint about the wing axis (sun
    tracking); each further segment hangs off the previous one by a fold
    joint about axis_across at their common edge.  Panels lie in the plane
    spanned by axis_along and axis_across.
    """
    along = np.asarray(axis_along, float) * sign
    across = np.asarray(axis_across, float)
    seg_len = length / n_segments
    parent = root
    for k in range(n_segments):
        pivot = along * (root_dist + k * seg_len)
        ax = axis_along if k == 0 else axis_across
        node = b.node(parent=parent, is_panel=1, pivot=tuple(pivot), axes=[ax],
                      lo=[-lim], hi=[lim])
        origin = pivot - across * (width / 2)
        b.quad_grid(origin, across * width, along * seg_len, nx, ny, node, mat_fn)
        parent = node


def procedural_spacecraft(seed=2, n_subboxes=40, dish_rings=64, dish_sectors=64,
                          seg_nx=40, seg_ny=64, n_segments=4, n_mats=6) -> Scene:
    """~50k-triangle procedural spacecraft.

    Bus [-1,1]^3 (12 tris); `n_subboxes` boxes with extents U(0.1,0.6) per axis
    centred on uniform points of random bus faces (half embedded); a 1.2 m
    paraboloid dish (focal 0.5 m, rings x sectors grid, two-sided single layer)
    above the +z face; two 8 m x 2.5 m wings along +-y from root hinges at
    y = +-1.5, each `n_segments` segments of seg_nx (x) by seg_ny (y) quads.
    Materials: n_mats pairs rho_s, rho_d ~ U(0,0.6) with rho_s + rho_d <= 0.9.
    Defaults give 12 + 480 + 8192 + 40960 = 49,644 triangles, 9 nodes, 8 DOF.
    """
    rng = np.random.default_rng(seed)
    mats = _random_mats(rng, n_mats)
    b = _Builder()
    root = b.node()
    b.box((0, 0, 0), (1, 1, 1), root, 0)
    for _ in range(n_subboxes):
        f = int(rng.integers(6))
        ax, sgn = f // 2, (1.0 if f % 2 else -1.0)
        c = rng.uniform(-1, 1, size=3)
        c[ax] = sgn
        ext = rng.uniform(0.1, 0.6, size=3)
        b.box(c, ext / 2, root, int(rng.integers(0, 3)) % n_mats)
    b.dish((0.0, 0.0), 1.35, 0.6, 0.5, dish_rings, dish_sectors, root, 3 % n_mats)
    m4, m5 = 4 % n_mats, 5 % n_mats
    for s in (1.0, -1.0):
        _panel_chain(b, root, s, (0, 1, 0), (1, 0, 0), 1.5, 8.0, 2.5, n_segments,
                     seg_nx, seg_ny, lambda a, c: np.where((a + c) % 2 == 0, m4, m5))
    return b.build(mats, name="procedural", meta=dict(seed=seed))


def procedural_sized(seed, target_tris) -> Scene:
    """The procedural generator with its tessellation scaled so that the
    triangle count is close to `target_tris` (used for uneven batches)."""
    s = np.sqrt(max(target_tris - 492, 64) / 49152.0)
    dr = max(3, int(round(64 * s)))
    nx = max(1, int(round(40 * s)))
    ny = max(1, int(round(64 * s)))
    return procedural_spacecraft(seed=seed, dish_rings=dr, dish_sectors=dr,
                                 seg_nx=nx, seg_ny=ny)


def uneven_batch_specs(seed=4, n=64):
    """Specs of an uneven batch: per item a triangle target log-uniform in
    [1e3, 5e5], a grid size 64*round(exp(U(ln 256, ln 2048))/64), root hinge
    angles U(-90,90) deg and a random sun direction."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        T = int(round(np.exp(rng.uniform(np.log(1e3), np.log(5e5)))))
        N = int(64 * round(np.exp(rng.uniform(np.log(256), np.log(2048))) / 64))
        ang = rng.uniform(-HALF_PI, HALF_PI, size=2)
        sun = rng.normal(size=3)
        out.append(dict(seed=seed * 1000 + k, target_tris=T, n=N, root_angles=ang,
                        sun_dir=sun / np.linalg.norm(sun)))
    return out


def greebled_spacecraft(seed=5, bus_n=160, n_greebles=2000, seg_nx=55, seg_ny=95,
                        n_segments=16, n_mats=8) -> Scene:
    """~1M-triangle procedural spacecraft: a 2 x 2 x 3 m bus whose faces are
    bus_n x bus_n quad grids, `n_greebles` small boxes (extents U(0.01,0.15))
    half embedded on random bus-face points, and four 16 m x 2 m wings along
    +-x and +-y, each `n_segments` segments of seg_nx x seg_ny quads
    (4 * n_segments degrees of freedom).  Defaults: 307,200 + 24,000 +
    668,800 = 1,000,000 triangles, 65 nodes, 64 DOF."""
    rng = np.random.default_rng(seed)
    mats = _random_mats(rng, n_mats)
    b = _Builder()
    root = b.node()
    half = np.array([1.0, 1.0, 1.5])
    for f in range(6):
        ax, sgn = f // 2, (1.0 if f % 2 else -1.0)
        o = -half.copy()
        o[ax] = sgn * half[ax]
        e = [np.zeros(3), np.zeros(3)]
        others = [a for a in range(3) if a != ax]
        e[0][others[0]] = 2 * half[others[0]]
        e[1][others[1]] = 2 * half[others[1]]
        b.quad_grid(o, e[0], e[1], bus_n, bus_n, root, lambda a, c, f=f: f % 2 + 0 * a)
    for _ in range(n_greebles):
        f = int(rng.integers(6))
        ax, sgn = f // 2, (1.0 if f % 2 else -1.0)
        c = rng.uniform(-1, 1, size=3) * half
        c[ax] = sgn * half[ax]
        ext = rng.uniform(0.01, 0.15, size=3)
        b.box(c, ext / 2, root, 2 + int(rng.integers(0, 3)))
    pm = lambda a, c: 5 + (a + c) % 3  # noqa: E731
    for along, across in (((0, 1, 0), (1, 0, 0)), ((1, 0, 0), (0, 1, 0))):
        for s in (1.0, -1.0):
            _panel_chain(b, root, s, along, across, 1.5, 16.0, 2.0, n_segments,
                         seg_nx, seg_ny, pm)
    return b.build(mats, name="greebled", meta=dict(seed=seed))


def merge_static(scene: Scene, world_tri_verts: np.ndarray, name="static", tri_mat=None) -> Scene:
    """A single-node scene whose triangles are the given corner positions
    (T,3,3) with the material table of `scene` and its per-triangle materials
    (or `tri_mat`); used to compare an articulated scene against the same
    geometry supplied pre-moved, or to add facets to a mesh."""
    w = np.asarray(world_tri_verts, np.float64).reshape(-1, 3, 3)
    T = w.shape[0]
    b = _Builder()
    root = b.node()
    b.tris(w.reshape(-1, 3), np.arange(3 * T).reshape(T, 3), root,
           scene.tri_mat if tri_mat is None else tri_mat)
    return b.build(scene.mats, name=name)
