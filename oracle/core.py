"""ctypes wrapper of the FP64 oracle (oracle.c) — TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, IEEE semantics, OpenMP over pixels)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                        "-ffp-contract=off", src, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


class _Scene(C.Structure):
    _fields_ = [("nv", C.c_int64), ("verts", C.c_void_p), ("nt", C.c_int64),
                ("tris", C.c_void_p), ("tri_mat", C.c_void_p), ("tri_node", C.c_void_p),
                ("nm", C.c_int32), ("mats", C.c_void_p), ("nn", C.c_int32),
                ("parent", C.c_void_p), ("pivot", C.c_void_p), ("n_axes", C.c_void_p),
                ("axes", C.c_void_p), ("lo", C.c_void_p), ("hi", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("sun_dir", C.c_double * 3), ("pressure", C.c_double), ("n", C.c_int32),
                ("bounces", C.c_int32), ("ref", C.c_double * 3), ("n_diffuse", C.c_int32),
                ("pad_", C.c_int32)]


class _Grid(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("v", C.c_double * 3), ("d", C.c_double * 3),
                ("umin", C.c_double), ("umax", C.c_double), ("vmin", C.c_double),
                ("vmax", C.c_double), ("hmin", C.c_double), ("wu", C.c_double),
                ("wv", C.c_double), ("L", C.c_double), ("a_pix", C.c_double), ("h0", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("force", C.c_double * 3), ("torque", C.c_double * 3), ("n_rays", C.c_int64),
                ("n_hits", C.c_int64), ("n_secondary", C.c_int64),
                ("n_secondary_hits", C.c_int64), ("n_diffuse", C.c_int64),
                ("n_diffuse_hits", C.c_int64), ("n_box_tests", C.c_int64), ("n_tri_tests", C.c_int64),
                ("grid", _Grid)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = C.CDLL(_SO)
        P = C.c_void_p
        _lib.orc_eval.argtypes = [P, P, P, C.c_int32, P, C.c_int64, P, P, P]
        _lib.orc_shade_frozen.argtypes = [P, P, P, P, P, P, P]
        _lib.orc_grid_of.argtypes = [P, P, P, P]
        _lib.orc_articulate.argtypes = [P, P, P]
        _lib.orc_node_transforms.argtypes = [P, P, P]
        _lib.orc_threads.restype = C.c_int32
        _lib.orc_diffuse_set.argtypes = [C.c_int32, P]
        _lib.orc_shade_frozen_dir.argtypes = [P, P, P, P, P, P, P]
        for f in ("orc_eval", "orc_shade_frozen", "orc_grid_of", "orc_articulate",
                  "orc_node_transforms", "orc_diffuse_set", "orc_shade_frozen_dir"):
            getattr(_lib, f).restype = C.c_int
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _SceneRef:
    """Keeps contiguous copies alive while the C struct points at them."""

    def __init__(self, s):
        self.keep = [np.ascontiguousarray(x, dtype=dt) for x, dt in (
            (s.verts, np.float64), (s.tris, np.int32), (s.tri_mat, np.int32),
            (s.tri_node, np.int32), (s.mats, np.float64), (s.parent, np.int32),
            (s.pivot, np.float64), (s.n_axes, np.int32), (s.axes, np.float64),
            (s.lo, np.float64), (s.hi, np.float64))]
        k = self.keep
        self.c = _Scene(k[0].shape[0], _ptr(k[0]), k[1].shape[0], _ptr(k[1]), _ptr(k[2]),
                        _ptr(k[3]), k[4].shape[0], _ptr(k[4]), k[5].shape[0], _ptr(k[5]),
                        _ptr(k[6]), _ptr(k[7]), _ptr(k[8]), _ptr(k[9]), _ptr(k[10]))


def _params(sun_dir, pressure, n, bounces, ref, diffuse=0):
    return _Params((C.c_double * 3)(*np.asarray(sun_dir, float)), float(pressure), int(n),
                   int(bounces), (C.c_double * 3)(*np.asarray(ref, float)), int(diffuse), 0)


def record_slots(bounces, diffuse=0):
    """Recorded hits per pixel: B + 1 chain generations, then the B diffuse
    fans of K rays (the fan of generation g at B + 1 + g K)."""
    return bounces + 1 + bounces * max(int(diffuse), 0)


@dataclass
class OracleResult:
    force: np.ndarray
    torque: np.ndarray
    n_rays: int
    n_hits: int
    n_secondary: int
    n_secondary_hits: int
    grid: dict
    ids: np.ndarray | None = None
    ts: np.ndarray | None = None
    n_diffuse: int = 0
    n_diffuse_hits: int = 0
    n_box_tests: int = 0
    n_tri_tests: int = 0


def _grid_dict(g: _Grid) -> dict:
    return dict(u=np.array(g.u[:]), v=np.array(g.v[:]), d=np.array(g.d[:]), umin=g.umin,
                umax=g.umax, vmin=g.vmin, vmax=g.vmax, hmin=g.hmin, wu=g.wu, wv=g.wv, L=g.L,
                a_pix=g.a_pix, h0=g.h0)


def _grid_struct(d: dict) -> _Grid:
    return _Grid((C.c_double * 3)(*d["u"]), (C.c_double * 3)(*d["v"]), (C.c_double * 3)(*d["d"]),
                 d["umin"], d["umax"], d["vmin"], d["vmax"], d["hmin"], d["wu"], d["wv"], d["L"],
                 d["a_pix"], d["h0"])


def _angles(scene, angles):
    if angles is None:
        return np.zeros(max(scene.n_dof, 1))
    a = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1)
    if a.shape[0] != scene.n_dof:
        raise ValueError(f"expected {scene.n_dof} angles, got {a.shape[0]}")
    return a if a.shape[0] else np.zeros(1)


def eval_srp(scene, sun_dir, n, bounces=0, pressure=1.0, ref=(0, 0, 0), angles=None,
             use_bvh=None, pixels=None, record=False, diffuse=0) -> OracleResult:
    """Force and torque of one evaluation (sum over all N*N pixels, or over
    the listed pixel indices p = j*N + i), with `diffuse` diffuse rays per
    emitting hit.  With record=True also returns the per-pixel hit ids and t
    of every ray, shape (n_pix, record_slots(bounces, diffuse))."""
    lib = _load()
    sr = _SceneRef(scene)
    ang = _angles(scene, angles)
    P = _params(sun_dir, pressure, n, bounces, ref, diffuse)
    if use_bvh is None:
        use_bvh = scene.n_tris > 64
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    npx = n * n if pix is None else pix.shape[0]
    G = record_slots(bounces, diffuse)
    ids = np.empty((npx, G), np.int32) if record else None
    ts = np.empty((npx, G), np.float64) if record else None
    out = _Result()
    rc = lib.orc_eval(C.byref(sr.c), _ptr(ang), C.byref(P), int(bool(use_bvh)), _ptr(pix),
                      npx, C.byref(out), _ptr(ids), _ptr(ts))
    if rc != 0:
        raise ValueError(f"oracle eval failed ({rc})")
    return OracleResult(np.array(out.force[:]), np.array(out.torque[:]), out.n_rays, out.n_hits,
                        out.n_secondary, out.n_secondary_hits, _grid_dict(out.grid), ids, ts,
                        out.n_diffuse, out.n_diffuse_hits, out.n_box_tests, out.n_tri_tests)


def diffuse_set(K) -> np.ndarray:
    """The K local diffuse directions (K, 3) in the hit's (t, b, n) frame."""
    lib = _load()
    out = np.empty((int(K), 3))
    if lib.orc_diffuse_set(int(K), _ptr(out)) != 0:
        raise ValueError("K must be >= 1")
    return out


def threads() -> int:
    """OpenMP threads the oracle's pixel loops use."""
    return int(_load().orc_threads())


def grid_of(scene, sun_dir, n, angles=None) -> dict:
    lib = _load()
    sr = _SceneRef(scene)
    g = _Grid()
    rc = lib.orc_grid_of(C.byref(sr.c), _ptr(_angles(scene, angles)),
                         C.byref(_params(sun_dir, 1.0, n, 0, (0, 0, 0))), C.byref(g))
    if rc != 0:
        raise ValueError(f"oracle grid failed ({rc})")
    return _grid_dict(g)


def articulate(scene, angles=None) -> np.ndarray:
    """Articulated triangle corners, shape (T, 3, 3)."""
    lib = _load()
    sr = _SceneRef(scene)
    w = np.empty((scene.n_tris, 3, 3))
    lib.orc_articulate(C.byref(sr.c), _ptr(_angles(scene, angles)), _ptr(w))
    return w


def node_transforms(scene, angles=None) -> np.ndarray:
    """Per-node rigid transforms (K, 3, 4): x_world = X[:, :3] x + X[:, 3]."""
    lib = _load()
    sr = _SceneRef(scene)
    xf = np.empty((scene.n_nodes, 12))
    lib.orc_node_transforms(C.byref(sr.c), _ptr(_angles(scene, angles)), _ptr(xf))
    return np.concatenate([xf[:, :9].reshape(-1, 3, 3), xf[:, 9:].reshape(-1, 3, 1)], axis=2)


def shade_frozen(scene, sun_dir, n, bounces, grid: dict, ids, pressure=1.0, ref=(0, 0, 0),
                 angles=None, diffuse=0, angles_ref=None) -> OracleResult:
    """Fixed-visibility re-shade of recorded rays (ids shape
    (N*N, record_slots(bounces, diffuse))).  With angles_ref (the angles the
    ids were recorded at) every primary ray keeps its share of its triangle's
    visible surface: its contribution scales with c0(angles)/c0(angles_ref)."""
    lib = _load()
    sr = _SceneRef(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32).reshape(n * n, record_slots(bounces, diffuse))
    g = _grid_struct(grid)
    out = _Result()
    aref = None if angles_ref is None else _angles(scene, angles_ref)
    rc = lib.orc_shade_frozen(C.byref(sr.c), _ptr(_angles(scene, angles)), _ptr(aref),
                              C.byref(_params(sun_dir, pressure, n, bounces, ref, diffuse)), C.byref(g),
                              _ptr(ids), C.byref(out))
    if rc != 0:
        raise ValueError(f"oracle shade failed ({rc})")
    return OracleResult(np.array(out.force[:]), np.array(out.torque[:]), out.n_rays, out.n_hits,
                        out.n_secondary, out.n_secondary_hits, grid, None, None, out.n_diffuse,
                        out.n_diffuse_hits)


def fd_gradients(scene, sun_dir, n, bounces, grid, ids, pressure=1.0, angles=None, h=1e-4,
                 which=("rho_s", "rho_d", "theta"), theta_idx=None, diffuse=0):
    """Central finite differences (FP64) of the fixed-visibility force with
    respect to each material's rho_s and rho_d and each hinge angle (or the
    hinges listed in theta_idx).  Every primary ray keeps its triangle and
    its share of that triangle's visible surface (shade_frozen with
    angles_ref = the recorded angles).  Returns dict name -> array (count, 3)."""
    ang = np.zeros(scene.n_dof) if angles is None else np.asarray(angles, float).copy()
    out = {}

    def F(sc, a):
        return shade_frozen(sc, sun_dir, n, bounces, grid, ids, pressure, (0, 0, 0), a, diffuse,
                            angles_ref=ang).force

    for col, name in ((0, "rho_s"), (1, "rho_d")):
        if name not in which:
            continue
        g = np.zeros((scene.n_mats, 3))
        for m in range(scene.n_mats):
            mp, mm = scene.mats.copy(), scene.mats.copy()
            mp[m, col] += h
            mm[m, col] -= h
            g[m] = (F(_unchecked(scene, mp), ang) - F(_unchecked(scene, mm), ang)) / (2 * h)
        out[name] = g
    if "theta" in which:
        idx = range(scene.n_dof) if theta_idx is None else list(theta_idx)
        g = np.zeros((len(idx), 3))
        for r, j in enumerate(idx):
            ap, am = ang.copy(), ang.copy()
            ap[j] += h
            am[j] -= h
            g[r] = (F(scene, ap) - F(scene, am)) / (2 * h)
        out["theta"] = g
    return out


def _unchecked(scene, mats):
    """Scene with stepped coefficients; the step must keep every material
    admissible (rho_s, rho_d >= 0, rho_s + rho_d <= 1)."""
    m = np.asarray(mats, float)
    if (m >= 0).all() and (m.sum(1) <= 1).all():
        return scene.with_mats(m)
    raise ValueError("finite-difference step leaves the admissible coefficient range; "
                     "use coefficients at least h inside [0,1]")


def shade_frozen_dir(scene, n, bounces, grid: dict, ids, dnew, pressure=1.0, angles=None):
    """Force of the recorded chains (ids (N*N, B+1)) when the photon direction
    becomes dnew, each primary ray keeping its triangle and its share of the
    triangle's visible area (scaled by c0(dnew)/c0(recorded))."""
    lib = _load()
    sr = _SceneRef(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32).reshape(n * n, bounces + 1)
    g = _grid_struct(grid)
    dn = np.ascontiguousarray(dnew, dtype=np.float64)
    out = _Result()
    rc = lib.orc_shade_frozen_dir(C.byref(sr.c), _ptr(_angles(scene, angles)),
                                  C.byref(_params(-grid["d"], pressure, n, bounces, (0, 0, 0))), C.byref(g),
                                  _ptr(ids), _ptr(dn), C.byref(out))
    if rc != 0:
        raise ValueError(f"oracle shade failed ({rc})")
    return np.array(out.force[:])


def fd_dir_jacobian(scene, n, bounces, grid, ids, pressure=1.0, angles=None, h=1e-6):
    """Central differences of shade_frozen_dir: J[i, j] = dF_i/dd_j at the
    recorded photon direction, d varied as a free 3-vector."""
    d0 = np.asarray(grid["d"], float)
    J = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (shade_frozen_dir(scene, n, bounces, grid, ids, d0 + e, pressure, angles) -
                   shade_frozen_dir(scene, n, bounces, grid, ids, d0 - e, pressure, angles)) / (2 * h)
    return J
