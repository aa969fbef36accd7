"""ctypes declarations of the C ABI in include/srp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsrp_mi355x.so")

SRP_OK, SRP_ERR_ARG, SRP_ERR_OOM, SRP_ERR_DEVICE, SRP_ERR_DEPTH = 0, -1, -2, -3, -4
SRP_F_COUNT = 1
SRP_MAX_N, SRP_MAX_BOUNCES, SRP_MAX_NODES, SRP_MAX_MATS, SRP_MAX_DIFFUSE = 8192, 4, 128, 64, 64

EXPORTS = [
    "srp_build_scene", "srp_destroy_scene", "srp_scene_n_dof", "srp_set_materials",
    "srp_set_panel_angles", "srp_eval", "srp_eval_batch", "srp_eval_batch_noalloc", "srp_eval_grad",
    "srp_eval_grad_batch", "srp_last_error", "srp_profile", "srp_profile_read", "srp_profile_read_launch",
    "srp_sun_tracking_angles", "srp_rk4", "srp_propagate",
    "srp_plan_create", "srp_plan_update", "srp_plan_launch", "srp_plan_destroy",
    "srp_set_schedule", "srp_autotune", "srp_spad_build", "srp_spad_interp", "srp_propagate_spad",
    "srp_rk78", "srp_propagate_rk78", "srp_propagate_spad_rk78",
    "srp_nplate_from_scene", "srp_nplate_from_mesh", "srp_nplate_eval", "srp_propagate_nplate",
    "srp_propagate_nplate_rk78", "srp_valu_peak",
]
SRP_PLAN_GRAD = 1
SRP_F_GRAD_DIR = 2


class srp_material(C.Structure):
    _fields_ = [("rho_s", C.c_double), ("rho_d", C.c_double)]


class srp_node(C.Structure):
    _fields_ = [("parent", C.c_int32), ("is_panel", C.c_int32), ("pivot", C.c_double * 3),
                ("n_axes", C.c_int32), ("reserved", C.c_int32), ("axis", (C.c_double * 3) * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class srp_eval_params(C.Structure):
    _fields_ = [("sun_dir", C.c_double * 3), ("pressure", C.c_double), ("n", C.c_int32),
                ("bounces", C.c_int32), ("ref", C.c_double * 3), ("flags", C.c_uint32),
                ("n_diffuse", C.c_int32)]


class srp_result(C.Structure):
    _fields_ = [("force", C.c_double * 3), ("torque", C.c_double * 3), ("n_rays", C.c_int64),
                ("n_hits", C.c_int64), ("n_secondary", C.c_int64),
                ("n_secondary_hits", C.c_int64), ("n_box_tests", C.c_int64),
                ("n_tri_tests", C.c_int64), ("status", C.c_uint32), ("n_clamped", C.c_uint32)]


class srp_batch_item(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("angles", C.c_void_p), ("p", srp_eval_params)]


class srp_orbit_params(C.Structure):
    _fields_ = [("mu", C.c_double), ("mass", C.c_double), ("p_ref", C.c_double),
                ("r_ref", C.c_double), ("n", C.c_int32), ("bounces", C.c_int32),
                ("track_sun", C.c_int32), ("n_diffuse", C.c_int32), ("ref", C.c_double * 3)]


class srp_spad_grid(C.Structure):
    _fields_ = [("n_az", C.c_int32), ("n_el", C.c_int32), ("az0", C.c_double), ("el0", C.c_double),
                ("daz", C.c_double), ("del_", C.c_double)]


class srp_plate(C.Structure):
    _fields_ = [("normal", C.c_double * 3), ("center", C.c_double * 3), ("area", C.c_double),
                ("rho_s", C.c_double), ("rho_d", C.c_double), ("two_sided", C.c_int32), ("reserved", C.c_int32)]


class srp_rk78_opts(C.Structure):
    _fields_ = [("h0", C.c_double), ("adaptive", C.c_int32), ("reserved", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double * 6), ("h_min", C.c_double), ("h_max", C.c_double)]


class srp_prop_stats(C.Structure):
    _fields_ = [("n_evals", C.c_int64), ("srp_seconds", C.c_double)]


ACCEL_FN = C.CFUNCTYPE(C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                       C.POINTER(C.c_double), C.c_void_p)

RESULT_DTYPE = np.dtype([("force", "<f8", 3), ("torque", "<f8", 3), ("n_rays", "<i8"),
                         ("n_hits", "<i8"), ("n_secondary", "<i8"), ("n_secondary_hits", "<i8"),
                         ("n_box_tests", "<i8"), ("n_tri_tests", "<i8"), ("status", "<u4"),
                         ("n_clamped", "<u4")])
assert RESULT_DTYPE.itemsize == C.sizeof(srp_result)

_lib = None


def load(path: str | None = None):
    """Loads the library.  torch is imported first so that the library binds
    to the HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (must precede the library: shared HIP runtime)
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2608_07307_amd.build` "
                           "(there is no CPU fallback)")
    lib = C.CDLL(p)
    V, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    lib.srp_build_scene.argtypes = [V, I64, V, I64, V, V, V, I32, V, I32, C.POINTER(V)]
    lib.srp_destroy_scene.argtypes = [V]
    lib.srp_scene_n_dof.argtypes = [V]
    lib.srp_scene_n_dof.restype = I32
    lib.srp_set_materials.argtypes = [V, V, I32]
    lib.srp_set_panel_angles.argtypes = [V, V, I32]
    lib.srp_eval.argtypes = [V, C.POINTER(srp_eval_params), C.POINTER(srp_result), V, V]
    lib.srp_eval_batch.argtypes = [V, I64, V, V]
    lib.srp_eval_batch_noalloc.argtypes = [V, I64, V, V]
    lib.srp_valu_peak.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(I32)]
    lib.srp_eval_grad.argtypes = [V, C.POINTER(srp_eval_params), C.POINTER(srp_result), V, V, V, V]
    lib.srp_eval_grad_batch.argtypes = [V, I64, V, V, I64, V]
    lib.srp_last_error.restype = C.c_char_p
    lib.srp_profile.argtypes = [C.c_int]
    lib.srp_sun_tracking_angles.argtypes = [V, V, V, I32]
    lib.srp_plan_create.argtypes = [V, I64, I32, V, V, I64, C.POINTER(V)]
    lib.srp_plan_update.argtypes = [V, V, I64]
    lib.srp_plan_launch.argtypes = [V, V]
    lib.srp_plan_destroy.argtypes = [V]
    lib.srp_set_schedule.argtypes = [I32, I32]
    lib.srp_autotune.argtypes = [V, I64, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(C.c_double)]
    lib.srp_rk4.argtypes = [V, C.c_double, C.c_double, I64, ACCEL_FN, V, V]
    lib.srp_propagate.argtypes = [V, C.POINTER(srp_orbit_params), V, V, C.c_double, C.c_double, I64, V,
                                  C.POINTER(srp_prop_stats)]
    lib.srp_profile_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.srp_profile_read_launch.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.srp_spad_build.argtypes = [V, C.POINTER(srp_eval_params), V, C.POINTER(srp_spad_grid), V]
    lib.srp_rk78.argtypes = [V, C.c_double, C.c_double, C.POINTER(srp_rk78_opts), ACCEL_FN, V, V, I64,
                             C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.srp_propagate_rk78.argtypes = [V, C.POINTER(srp_orbit_params), V, V, C.c_double, C.c_double,
                                       C.POINTER(srp_rk78_opts), V, I64, C.POINTER(C.c_int64),
                                       C.POINTER(srp_prop_stats)]
    lib.srp_propagate_spad_rk78.argtypes = [C.POINTER(srp_spad_grid), V, C.c_double, C.POINTER(srp_orbit_params),
                                            V, C.c_double, C.c_double, C.POINTER(srp_rk78_opts), V, I64,
                                            C.POINTER(C.c_int64)]
    lib.srp_spad_interp.argtypes = [C.POINTER(srp_spad_grid), V, V, V]
    lib.srp_nplate_from_scene.argtypes = [V, V, V, C.c_int32, C.POINTER(C.c_int32)]
    lib.srp_nplate_from_mesh.argtypes = [V, I64, V, I64, V, V, V, I32, V, I32, V, V, C.c_int32,
                                         C.POINTER(C.c_int32)]
    lib.srp_nplate_eval.argtypes = [V, C.c_int32, V, C.c_double, V, V, V]
    lib.srp_propagate_nplate.argtypes = [V, C.c_int32, C.POINTER(srp_orbit_params), V, C.c_double, C.c_double,
                                         I64, V]
    lib.srp_propagate_nplate_rk78.argtypes = [V, C.c_int32, C.POINTER(srp_orbit_params), V, C.c_double,
                                              C.c_double, C.POINTER(srp_rk78_opts), V, I64, C.POINTER(C.c_int64)]
    lib.srp_propagate_spad.argtypes = [C.POINTER(srp_spad_grid), V, C.c_double, C.POINTER(srp_orbit_params), V,
                                       C.c_double, C.c_double, I64, V]
    for f in ("srp_build_scene", "srp_destroy_scene", "srp_set_materials",
              "srp_set_panel_angles", "srp_eval", "srp_eval_batch", "srp_eval_batch_noalloc", "srp_eval_grad",
              "srp_eval_grad_batch", "srp_profile", "srp_profile_read", "srp_profile_read_launch",
              "srp_sun_tracking_angles", "srp_rk4", "srp_propagate", "srp_plan_create",
              "srp_plan_update", "srp_plan_launch", "srp_plan_destroy", "srp_set_schedule",
              "srp_autotune", "srp_spad_build", "srp_spad_interp", "srp_propagate_spad", "srp_rk78",
              "srp_propagate_rk78", "srp_propagate_spad_rk78", "srp_nplate_from_scene", "srp_nplate_eval",
              "srp_nplate_from_mesh", "srp_propagate_nplate", "srp_propagate_nplate_rk78"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


class SrpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"srp error {code}: {msg}")
        self.code = code


def check(rc: int) -> int:
    if rc < 0:
        raise SrpError(rc, _lib.srp_last_error().decode())
    return rc


def ptr(a) -> C.c_void_p | None:
    if a is None:
        return None
    return C.c_void_p(a.ctypes.data)
