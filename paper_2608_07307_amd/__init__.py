"""MI355X-native ray-traced solar-radiation-pressure (SRP) library.

Python binding of the C ABI in include/srp.h.  Every step of an evaluation
runs in the gfx950 kernels of libsrp_mi355x.so; this module only marshals
arguments (numpy arrays, torch device tensors and HIP streams).  There is no
CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import RESULT_DTYPE, SRP_F_COUNT, SrpError  # noqa: F401

__all__ = ["Scene", "params", "eval", "eval_grad", "Batch", "eval_batch", "eval_grad_batch",
           "PLATE_DTYPE", "nplate_from_scene", "nplate_from_mesh", "nplate_eval", "propagate_nplate", "propagate_nplate_rk78",
           "SrpError", "RESULT_DTYPE"]


def _load():
    return L.load()


def params(sun_dir, n, bounces=0, pressure=1.0, ref=(0.0, 0.0, 0.0), count=False, diffuse=0, grad_dir=False):
    p = L.srp_eval_params()
    p.sun_dir[:] = [float(x) for x in sun_dir]
    p.pressure = float(pressure)
    p.n = int(n)
    p.bounces = int(bounces)
    p.ref[:] = [float(x) for x in ref]
    p.flags = (L.SRP_F_COUNT if count else 0) | (L.SRP_F_GRAD_DIR if grad_dir else 0)
    p.n_diffuse = int(diffuse)
    return p


def record_slots(bounces, diffuse=0):
    """Recorded rays per pixel: B + 1 chain generations, then B fans of K
    diffuse rays (generation g's fan at B + 1 + g K)."""
    return int(bounces) + 1 + int(bounces) * int(diffuse)


def _mesh_arrays(mesh):
    """The arrays srp_build_scene takes, from a mesh object (see Scene)."""
    verts = np.ascontiguousarray(mesh.verts, dtype=np.float64)
    tris = np.ascontiguousarray(mesh.tris, dtype=np.int32)
    tm = np.ascontiguousarray(mesh.tri_mat, dtype=np.int32)
    tn = np.ascontiguousarray(mesh.tri_node, dtype=np.int32)
    mats = (L.srp_material * len(mesh.mats))(*[L.srp_material(float(a), float(b)) for a, b in mesh.mats])
    K = len(mesh.parent)
    nodes = (L.srp_node * K)()
    for k in range(K):
        nd = nodes[k]
        nd.parent = int(mesh.parent[k])
        nd.is_panel = int(mesh.is_panel[k])
        nd.pivot[:] = [float(x) for x in mesh.pivot[k]]
        nd.n_axes = int(mesh.n_axes[k])
        for a in range(3):
            nd.axis[a][:] = [float(x) for x in mesh.axes[k][a]]
        nd.lo[:] = [float(x) for x in mesh.lo[k]]
        nd.hi[:] = [float(x) for x in mesh.hi[k]]
    return verts, tris, tm, tn, mats, nodes


class Scene:
    """A scene built by srp_build_scene from mesh, materials and tree arrays.

    `mesh` is any object with the attributes verts (V,3), tris (T,3),
    tri_mat (T,), tri_node (T,), mats (M,2), parent, is_panel, pivot,
    n_axes, axes (K,3,3), lo, hi (K,3)."""

    def __init__(self, mesh):
        lib = _load()
        verts, tris, tm, tn, mats, nodes = _mesh_arrays(mesh)
        K = len(nodes)
        h = C.c_void_p()
        L.check(lib.srp_build_scene(L.ptr(verts), verts.shape[0], L.ptr(tris), tris.shape[0],
                                    L.ptr(tm), L.ptr(tn), mats, len(mesh.mats), nodes, K,
                                    C.byref(h)))
        self.handle = h
        self.n_dof = int(lib.srp_scene_n_dof(h))
        self.n_mats = len(mesh.mats)
        self.n_nodes = K
        self.n_tris = tris.shape[0]

    def close(self):
        if getattr(self, "handle", None) is not None and L._lib is not None:
            L._lib.srp_destroy_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_angles(self, angles) -> int:
        a = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1)
        return L.check(_load().srp_set_panel_angles(self.handle, L.ptr(a) if a.size else None, a.size))

    def set_materials(self, mats):
        m = np.asarray(mats, dtype=np.float64).reshape(-1, 2)
        arr = (L.srp_material * len(m))(*[L.srp_material(float(a), float(b)) for a, b in m])
        L.check(_load().srp_set_materials(self.handle, arr, len(m)))


def _result_dict(r) -> dict:
    return dict(force=np.array(r.force[:]), torque=np.array(r.torque[:]), n_rays=r.n_rays,
                n_hits=r.n_hits, n_secondary=r.n_secondary, n_secondary_hits=r.n_secondary_hits,
                n_box_tests=r.n_box_tests, n_tri_tests=r.n_tri_tests, status=r.status, n_clamped=r.n_clamped)


def eval(scene: Scene, sun_dir, n, bounces=0, pressure=1.0, ref=(0, 0, 0), count=False,
         record=False, diffuse=0) -> dict:
    """srp_eval at the scene's current angles with `diffuse` diffuse rays per
    emitting hit.  With record=True the result also holds ids (N*N, R) int32
    and ts (N*N, R) float32, R = record_slots(bounces, diffuse)."""
    lib = _load()
    p = params(sun_dir, n, bounces, pressure, ref, count, diffuse)
    r = L.srp_result()
    ids = ts = None
    if record:
        R = record_slots(bounces, diffuse)
        ids = np.empty((n * n, R), np.int32)
        ts = np.empty((n * n, R), np.float32)
    L.check(lib.srp_eval(scene.handle, C.byref(p), C.byref(r), L.ptr(ids), L.ptr(ts)))
    out = _result_dict(r)
    if record:
        out["ids"], out["ts"] = ids, ts
    return out


def eval_grad(scene: Scene, sun_dir, n, bounces=0, pressure=1.0, ref=(0, 0, 0)) -> dict:
    """srp_eval_grad: result plus dF/drho_s (M,3), dF/drho_d (M,3), dF/dtheta (J,3)
    and dF/dd (3,3), d the photon direction."""
    lib = _load()
    p = params(sun_dir, n, bounces, pressure, ref)
    r = L.srp_result()
    gs = np.zeros((scene.n_mats, 3))
    gd = np.zeros((scene.n_mats, 3))
    gt = np.zeros((max(scene.n_dof, 1), 3))
    gdir = np.zeros((3, 3))
    L.check(lib.srp_eval_grad(scene.handle, C.byref(p), C.byref(r), L.ptr(gs), L.ptr(gd), L.ptr(gt), L.ptr(gdir)))
    out = _result_dict(r)
    out.update(rho_s=gs, rho_d=gd, theta=gt[: scene.n_dof], dir=gdir)
    return out


def grad_size(scene: Scene) -> int:
    """Gradient doubles of one evaluation: 3 (2M + J) + 9."""
    return 3 * (2 * scene.n_mats + scene.n_dof) + 9


class Batch:
    """A batch marshalled once into its srp_batch_item array, for repeated
    launches (eval_batch / eval_grad_batch accept it in place of the entry
    list).  Holds the scenes and angle arrays the items point to."""

    def __init__(self, entries):
        self.entries = list(entries)
        self.arr, self.keep = _items(self.entries)

    def __len__(self):
        return len(self.entries)


def _marshalled(entries):
    """(item array, objects it points into, n) for an entry list or a Batch."""
    if isinstance(entries, Batch):
        return entries.arr, entries.keep, len(entries)
    arr, keep = _items(entries)
    return arr, keep, len(entries)


def _items(entries):
    """entries: list of (scene, angles or None, params)."""
    arr = (L.srp_batch_item * len(entries))()
    keep = []
    for k, (sc, ang, p) in enumerate(entries):
        arr[k].scene = sc.handle
        if ang is not None:
            a = np.ascontiguousarray(ang, dtype=np.float64).reshape(-1)
            if a.size != sc.n_dof:
                raise ValueError("angles length differs from the scene's n_dof")
            keep.append(a)
            arr[k].angles = a.ctypes.data if a.size else None
        else:
            arr[k].angles = None
        arr[k].p = p
    return arr, keep


def eval_batch(entries, out=None, stream=None):
    """srp_eval_batch.  entries: list of (scene, angles or None, params), or a
    Batch.  Returns a uint8 device tensor of len(entries) srp_result records
    (use results_to_numpy to read it); stream-ordered on `stream` (torch
    stream)."""
    import torch
    lib = _load()
    arr, keep, n = _marshalled(entries)
    if out is None:
        out = torch.empty(n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    L.check(lib.srp_eval_batch(arr, n, C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)))
    return out


def valu_peak() -> dict:
    """srp_valu_peak: measured non-packed FP32 FMA issue rate (lane-FMAs/s),
    the shader clock it ran at (GHz) and the compute-unit count."""
    r, g, n = C.c_double(0), C.c_double(0), C.c_int32(0)
    L.check(_load().srp_valu_peak(C.byref(r), C.byref(g), C.byref(n)))
    return dict(lane_fma_per_s=r.value, shader_ghz=g.value, n_cu=n.value)


def eval_batch_noalloc(entries, out=None, stream=None):
    """srp_eval_batch_noalloc: srp_eval_batch through the library's fixed
    per-GPU workspace (the call allocates nothing; batches that do not fit are
    rejected).  Same arguments and result as eval_batch."""
    import torch
    lib = _load()
    arr, keep, n = _marshalled(entries)
    if out is None:
        out = torch.empty(n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    L.check(lib.srp_eval_batch_noalloc(arr, n, C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)))
    return out


def eval_grad_batch(entries, out=None, grad=None, stream=None):
    """srp_eval_grad_batch (entries: a list as for eval_batch, or a Batch).  Returns (results uint8 tensor, gradients float64
    tensor (n, stride)) with stride = max over entries of grad_size(scene):
    rho_s (M x 3), rho_d (M x 3), theta (J x 3), dF/dd (3 x 3) per row."""
    import torch
    lib = _load()
    arr, keep, n = _marshalled(entries)
    if out is None:
        out = torch.empty(n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    if grad is None:
        lst = entries.entries if isinstance(entries, Batch) else entries
        stride = max(grad_size(sc) for sc, _, _ in lst)
        grad = torch.zeros((n, stride), dtype=torch.float64, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    L.check(lib.srp_eval_grad_batch(arr, n, C.c_void_p(out.data_ptr()),
                                    C.c_void_p(grad.data_ptr()), grad.shape[1],
                                    C.c_void_p(s.cuda_stream)))
    return out, grad


def results_to_numpy(t) -> np.ndarray:
    """Structured array (RESULT_DTYPE) from a results tensor."""
    b = t.detach().cpu().numpy().tobytes()
    return np.frombuffer(b, dtype=RESULT_DTYPE)


def profile(enable: bool):
    """Start (True) or stop (False) timing trace-kernel launches; resets totals."""
    L.check(_load().srp_profile(1 if enable else 0))


def profile_read():
    """(summed milliseconds of the ray-tracing kernels, launch count) since the last reset."""
    ms, n = C.c_double(), C.c_int64()
    L.check(_load().srp_profile_read(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def profile_read_launch():
    """(summed milliseconds of whole launches: upload, every kernel, result copy; launch count)
    since the last reset."""
    ms, n = C.c_double(), C.c_int64()
    L.check(_load().srp_profile_read_launch(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def sun_tracking_angles(scene: Scene, sun_dir, angles=None) -> np.ndarray:
    """srp_sun_tracking_angles: wing roots turned towards the Sun (host)."""
    a = np.zeros(scene.n_dof) if angles is None else np.array(angles, dtype=np.float64)
    s = np.ascontiguousarray(sun_dir, dtype=np.float64)
    L.check(_load().srp_sun_tracking_angles(scene.handle, L.ptr(s), L.ptr(a) if a.size else None,
                                            a.size))
    return a


def rk4(y0, t0, h, n_steps, accel) -> np.ndarray:
    """srp_rk4 with a Python acceleration accel(t, r, v) -> a (host only)."""
    err = []

    def cb(t, r, v, a, _):
        try:
            out = accel(t, np.ctypeslib.as_array(r, (3,)).copy(), np.ctypeslib.as_array(v, (3,)).copy())
            for i in range(3):
                a[i] = float(out[i])
            return 0
        except Exception as e:  # reported after the call
            err.append(e)
            return -1

    f = L.ACCEL_FN(cb)
    y = np.ascontiguousarray(y0, dtype=np.float64)
    traj = np.zeros((n_steps + 1, 7))
    rc = _load().srp_rk4(L.ptr(y), float(t0), float(h), int(n_steps), f, None, L.ptr(traj))
    if err:
        raise err[0]
    L.check(rc)
    return traj


def propagate(scene: Scene, y0, t0, h, n_steps, mu, mass, p_ref, r_ref, n, bounces=0,
              track_sun=False, angles0=None, ref=(0.0, 0.0, 0.0), diffuse=0):
    """srp_propagate: heliocentric two-body + ray-traced SRP, RK4, one GPU
    evaluation per stage.  Returns (traj (n_steps+1, 7), stats dict)."""
    op = L.srp_orbit_params(float(mu), float(mass), float(p_ref), float(r_ref), int(n), int(bounces),
                            1 if track_sun else 0, int(diffuse), (C.c_double * 3)(*ref))
    y = np.ascontiguousarray(y0, dtype=np.float64)
    a0 = None if angles0 is None else np.ascontiguousarray(angles0, dtype=np.float64)
    traj = np.zeros((n_steps + 1, 7))
    st = L.srp_prop_stats()
    L.check(_load().srp_propagate(scene.handle, C.byref(op), L.ptr(a0) if a0 is not None and a0.size else None,
                                  L.ptr(y), float(t0), float(h), int(n_steps), L.ptr(traj), C.byref(st)))
    return traj, dict(n_evals=st.n_evals, srp_seconds=st.srp_seconds)


def rk78_opts(h0, adaptive=False, rtol=0.0, atol=(0.0,) * 6, h_min=0.0, h_max=0.0):
    """srp_rk78_opts: fixed steps h0, or adaptive with tolerances rtol and
    atol (6 values or one for all)."""
    a = np.broadcast_to(np.asarray(atol, dtype=np.float64), (6,))
    return L.srp_rk78_opts(float(h0), 1 if adaptive else 0, 0, float(rtol), (C.c_double * 6)(*a), float(h_min),
                           float(h_max))


def rk78(y0, t0, t1, accel, opts, max_rows=1 << 16):
    """srp_rk78 with a Python acceleration accel(t, r, v) -> a (host only).
    Returns (rows (t, y) of the accepted steps, derivative evaluations)."""
    err = []

    def cb(t, r, v, a, _):
        try:
            out = accel(t, np.ctypeslib.as_array(r, (3,)).copy(), np.ctypeslib.as_array(v, (3,)).copy())
            for i in range(3):
                a[i] = float(out[i])
            return 0
        except Exception as e:  # reported after the call
            err.append(e)
            return -1

    f = L.ACCEL_FN(cb)
    y = np.ascontiguousarray(y0, dtype=np.float64)
    traj = np.zeros((max_rows, 7))
    rows, evals = C.c_int64(0), C.c_int64(0)
    rc = _load().srp_rk78(L.ptr(y), float(t0), float(t1), C.byref(opts), f, None, L.ptr(traj), int(max_rows),
                          C.byref(rows), C.byref(evals))
    if err:
        raise err[0]
    L.check(rc)
    return traj[:rows.value].copy(), evals.value


def propagate_rk78(scene: Scene, y0, t0, t1, opts, mu, mass, p_ref, r_ref, n, bounces=0, track_sun=False,
                   angles0=None, ref=(0.0, 0.0, 0.0), diffuse=0, max_rows=1 << 16):
    """srp_propagate_rk78: two-body + ray-traced SRP with RK7(8), one GPU
    evaluation per stage.  Returns (rows (t, r, v), stats dict)."""
    op = L.srp_orbit_params(float(mu), float(mass), float(p_ref), float(r_ref), int(n), int(bounces),
                            1 if track_sun else 0, int(diffuse), (C.c_double * 3)(*ref))
    y = np.ascontiguousarray(y0, dtype=np.float64)
    a0 = None if angles0 is None else np.ascontiguousarray(angles0, dtype=np.float64)
    traj = np.zeros((max_rows, 7))
    rows = C.c_int64(0)
    st = L.srp_prop_stats()
    L.check(_load().srp_propagate_rk78(scene.handle, C.byref(op), L.ptr(a0) if a0 is not None and a0.size else None,
                                       L.ptr(y), float(t0), float(t1), C.byref(opts), L.ptr(traj), int(max_rows),
                                       C.byref(rows), C.byref(st)))
    return traj[:rows.value].copy(), dict(n_evals=st.n_evals, srp_seconds=st.srp_seconds)


def propagate_spad_rk78(grid, table, p_table, y0, t0, t1, opts, mu, mass, p_ref, r_ref, max_rows=1 << 16):
    """srp_propagate_spad_rk78.  Returns rows (t, r, v) of the accepted steps."""
    op = L.srp_orbit_params(float(mu), float(mass), float(p_ref), float(r_ref), 0, 0, 0, 0,
                            (C.c_double * 3)(0.0, 0.0, 0.0))
    t = np.ascontiguousarray(table, dtype=np.float64)
    y = np.ascontiguousarray(y0, dtype=np.float64)
    traj = np.zeros((max_rows, 7))
    rows = C.c_int64(0)
    L.check(_load().srp_propagate_spad_rk78(C.byref(grid), L.ptr(t), float(p_table), C.byref(op), L.ptr(y),
                                            float(t0), float(t1), C.byref(opts), L.ptr(traj), int(max_rows),
                                            C.byref(rows)))
    return traj[:rows.value].copy()


def spad_grid(n_az, n_el, az0, el0, daz, de):
    """srp_spad_grid (angles in radians)."""
    return L.srp_spad_grid(int(n_az), int(n_el), float(az0), float(el0), float(daz), float(de))


def spad_build(scene: Scene, grid, n, bounces=0, pressure=1.0, ref=(0.0, 0.0, 0.0), angles=None, diffuse=0):
    """srp_spad_build: (n_el, n_az, 6) force and torque at every grid direction."""
    tab = np.zeros((grid.n_el, grid.n_az, 6))
    p = params((1.0, 0.0, 0.0), n, bounces, pressure, ref, False, diffuse)
    a = None if angles is None else np.ascontiguousarray(angles, dtype=np.float64)
    L.check(_load().srp_spad_build(scene.handle, C.byref(p), L.ptr(a) if a is not None and a.size else None,
                                   C.byref(grid), L.ptr(tab)))
    return tab


def spad_interp(grid, table, sun_dir) -> np.ndarray:
    """srp_spad_interp: interpolated (force, torque) at a Sun direction."""
    t = np.ascontiguousarray(table, dtype=np.float64)
    s = np.ascontiguousarray(sun_dir, dtype=np.float64)
    out = np.zeros(6)
    L.check(_load().srp_spad_interp(C.byref(grid), L.ptr(t), L.ptr(s), L.ptr(out)))
    return out


def propagate_spad(grid, table, p_table, y0, t0, h, n_steps, mu, mass, p_ref, r_ref):
    """srp_propagate_spad: RK4 two-body + SRP interpolated from a SPAD table
    (built at pressure p_table).  Returns traj (n_steps+1, 7)."""
    op = L.srp_orbit_params(float(mu), float(mass), float(p_ref), float(r_ref), 0, 0, 0, 0,
                            (C.c_double * 3)(0.0, 0.0, 0.0))
    t = np.ascontiguousarray(table, dtype=np.float64)
    y = np.ascontiguousarray(y0, dtype=np.float64)
    traj = np.zeros((n_steps + 1, 7))
    L.check(_load().srp_propagate_spad(C.byref(grid), L.ptr(t), float(p_table), C.byref(op), L.ptr(y), float(t0),
                                       float(h), int(n_steps), L.ptr(traj)))
    return traj


PLATE_DTYPE = np.dtype([("normal", "<f8", 3), ("center", "<f8", 3), ("area", "<f8"), ("rho_s", "<f8"),
                        ("rho_d", "<f8"), ("two_sided", "<i4"), ("reserved", "<i4")])


def _plates(plates) -> np.ndarray:
    a = np.ascontiguousarray(plates, dtype=PLATE_DTYPE)
    return a


def _angle_vector(angles, n_dof) -> np.ndarray:
    """Hinge angles as a contiguous FP64 vector of exactly n_dof entries (the
    library reads that many)."""
    a = np.ascontiguousarray(angles, dtype=np.float64).reshape(-1)
    if a.shape[0] != n_dof:
        raise SrpError(-1, f"expected {n_dof} hinge angles, got {a.shape[0]}")
    return a


def nplate_from_scene(scene: Scene, angles=None) -> np.ndarray:
    """srp_nplate_from_scene: the scene's plates (PLATE_DTYPE records) at
    `angles` (None = its current angles)."""
    lib = _load()
    a = None if angles is None else _angle_vector(angles, scene.n_dof)
    n = C.c_int32(0)
    rc = lib.srp_nplate_from_scene(scene.handle, L.ptr(a) if a is not None else None, None, 0, C.byref(n))
    if rc != 0 and n.value == 0:
        L.check(rc)
    out = np.zeros(n.value, PLATE_DTYPE)
    L.check(lib.srp_nplate_from_scene(scene.handle, L.ptr(a) if a is not None else None,
                                      out.ctypes.data if n.value else None, n.value, C.byref(n)))
    return out


def nplate_from_mesh(mesh, angles=None) -> np.ndarray:
    """srp_nplate_from_mesh: the plates srp_nplate_from_scene would give for
    this mesh at `angles` (None = all zero), without a scene or a GPU."""
    lib = _load()
    verts, tris, tm, tn, mats, nodes = _mesh_arrays(mesh)
    a = None if angles is None else _angle_vector(angles, int(np.asarray(mesh.n_axes).sum()))
    args = (L.ptr(verts), verts.shape[0], L.ptr(tris), tris.shape[0], L.ptr(tm), L.ptr(tn), mats, len(mesh.mats),
            nodes, len(nodes), L.ptr(a) if a is not None else None)
    n = C.c_int32(0)
    rc = lib.srp_nplate_from_mesh(*args, None, 0, C.byref(n))
    if rc != 0 and n.value == 0:
        L.check(rc)
    out = np.zeros(n.value, PLATE_DTYPE)
    L.check(lib.srp_nplate_from_mesh(*args, out.ctypes.data if n.value else None, n.value, C.byref(n)))
    return out


def nplate_eval(plates, sun_dir, pressure=1.0, ref=(0.0, 0.0, 0.0)) -> dict:
    """srp_nplate_eval: N-plate force and torque."""
    p = _plates(plates)
    s = np.ascontiguousarray(sun_dir, dtype=np.float64)
    r = np.ascontiguousarray(ref, dtype=np.float64)
    f, t = np.zeros(3), np.zeros(3)
    L.check(_load().srp_nplate_eval(p.ctypes.data if len(p) else None, len(p), L.ptr(s), float(pressure),
                                    L.ptr(r), L.ptr(f), L.ptr(t)))
    return dict(force=f, torque=t)


def propagate_nplate(plates, y0, t0, h, n_steps, mu, mass, p_ref, r_ref):
    """srp_propagate_nplate: RK4 two-body + N-plate SRP, attitude fixed.
    Returns traj (n_steps+1, 7)."""
    p = _plates(plates)
    op = L.srp_orbit_params(float(mu), float(mass), float(p_ref), float(r_ref), 0, 0, 0, 0,
                            (C.c_double * 3)(0.0, 0.0, 0.0))
    y = np.ascontiguousarray(y0, dtype=np.float64)
    traj = np.zeros((n_steps + 1, 7))
    L.check(_load().srp_propagate_nplate(p.ctypes.data if len(p) else None, len(p), C.byref(op), L.ptr(y),
                                         float(t0), float(h), int(n_steps), L.ptr(traj)))
    return traj


def propagate_nplate_rk78(plates, y0, t0, t1, opts, mu, mass, p_ref, r_ref, max_rows=1 << 16):
    """srp_propagate_nplate_rk78.  Returns rows (t, r, v) of the accepted steps."""
    p = _plates(plates)
    op = L.srp_orbit_params(float(mu), float(mass), float(p_ref), float(r_ref), 0, 0, 0, 0,
                            (C.c_double * 3)(0.0, 0.0, 0.0))
    y = np.ascontiguousarray(y0, dtype=np.float64)
    traj = np.zeros((max_rows, 7))
    rows = C.c_int64(0)
    L.check(_load().srp_propagate_nplate_rk78(p.ctypes.data if len(p) else None, len(p), C.byref(op), L.ptr(y),
                                              float(t0), float(t1), C.byref(opts), L.ptr(traj), int(max_rows),
                                              C.byref(rows)))
    return traj[:rows.value].copy()


def set_schedule(patches_per_chunk=0, blocks_per_cu=0):
    """srp_set_schedule (0 = automatic)."""
    L.check(_load().srp_set_schedule(int(patches_per_chunk), int(blocks_per_cu)))


def autotune(entries, grad=False):
    """srp_autotune over a batch (entry list or Batch); returns
    (patches_per_chunk, blocks_per_cu, ms)."""
    arr, keep, n = _marshalled(entries)
    r, b, ms = C.c_int32(), C.c_int32(), C.c_double()
    L.check(_load().srp_autotune(arr, n, L.SRP_PLAN_GRAD if grad else 0, C.byref(r),
                                 C.byref(b), C.byref(ms)))
    return r.value, b.value, ms.value


class Plan:
    """srp_plan: a captured batch launch replayed with new per-item values."""

    def __init__(self, entries, grad=False):
        import torch
        n = len(entries)
        self.n = n
        self.out = torch.empty(n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self.stride = max(grad_size(sc) for sc, _, _ in entries)
        self.grad = torch.zeros((n, self.stride), dtype=torch.float64, device="cuda") if grad else None
        arr, keep = _items(entries)
        h = C.c_void_p()
        L.check(_load().srp_plan_create(arr, n, L.SRP_PLAN_GRAD if grad else 0,
                                        C.c_void_p(self.out.data_ptr()),
                                        C.c_void_p(self.grad.data_ptr()) if grad else None,
                                        self.stride, C.byref(h)))
        self.handle = h

    def update(self, entries):
        arr, keep = _items(entries)
        L.check(_load().srp_plan_update(self.handle, arr, len(entries)))

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        L.check(_load().srp_plan_launch(self.handle, C.c_void_p(s.cuda_stream)))
        return self.out

    def close(self):
        if getattr(self, "handle", None) is not None and L._lib is not None:
            L._lib.srp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
