"""C-ABI checks that need no GPU: the library loads, exports every function
include/srp.h declares, its public structs have the layout the binding
assumes, and invalid inputs are rejected before any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(srp_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_07307_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libsrp_mi355x.so is not built (run __graft_entry__.build())")
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 10, names
    from paper_2608_07307_amd import _lib as L
    assert sorted(L.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_binding(tmp_path):
    from paper_2608_07307_amd import _lib as L
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "srp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(srp_material), sizeof(srp_node), sizeof(srp_eval_params),
         sizeof(srp_result), sizeof(srp_batch_item));
  printf("%zu %zu %zu %zu\\n", offsetof(srp_node, axis), offsetof(srp_eval_params, flags),
         offsetof(srp_result, status), offsetof(srp_batch_item, p));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:2]
    sizes = [int(x) for x in a.split()]
    offs = [int(x) for x in b.split()]
    assert sizes == [C.sizeof(L.srp_material), C.sizeof(L.srp_node), C.sizeof(L.srp_eval_params),
                     C.sizeof(L.srp_result), C.sizeof(L.srp_batch_item)]
    assert offs == [L.srp_node.axis.offset, L.srp_eval_params.flags.offset,
                    L.srp_result.status.offset, L.srp_batch_item.p.offset]
    assert L.RESULT_DTYPE.itemsize == sizes[3]


def _build(lib, mesh, **over):
    from paper_2608_07307_amd import Scene  # noqa: F401
    from paper_2608_07307_amd import _lib as L
    d = dict(verts=np.ascontiguousarray(mesh.verts, np.float64),
             tris=np.ascontiguousarray(mesh.tris, np.int32),
             tm=np.ascontiguousarray(mesh.tri_mat, np.int32),
             tn=np.ascontiguousarray(mesh.tri_node, np.int32),
             mats=np.asarray(mesh.mats, float), parent=mesh.parent, n_axes=mesh.n_axes,
             lo=mesh.lo, hi=mesh.hi, axes=mesh.axes)
    d.update(over)
    mats = (L.srp_material * len(d["mats"]))(*[L.srp_material(*m) for m in d["mats"]])
    K = len(d["parent"])
    nodes = (L.srp_node * K)()
    for k in range(K):
        nodes[k].parent = int(d["parent"][k])
        nodes[k].n_axes = int(d["n_axes"][k])
        for a in range(3):
            nodes[k].axis[a][:] = list(map(float, d["axes"][k][a]))
        nodes[k].lo[:] = list(map(float, d["lo"][k]))
        nodes[k].hi[:] = list(map(float, d["hi"][k]))
    h = C.c_void_p()
    rc = lib.srp_build_scene(L.ptr(d["verts"]), d["verts"].shape[0], L.ptr(d["tris"]),
                             d["tris"].shape[0], L.ptr(d["tm"]), L.ptr(d["tn"]), mats,
                             len(d["mats"]), nodes, K, C.byref(h))
    return rc, lib.srp_last_error().decode(), h


@pytest.mark.parametrize("case", [
    "bad_vertex_index", "bad_material_index", "bad_node_index", "rho_sum_above_one",
    "negative_rho", "root_with_parent", "parent_not_before_child", "too_many_axes",
    "nan_vertex", "zero_axis", "inverted_interval",
])
def test_build_scene_rejects_invalid_input(lib, case):
    """Every invalid input returns SRP_ERR_ARG with a message and no handle,
    before any device work (so this runs on a machine without a GPU)."""
    m = synth.box_wing()
    over = {}
    if case == "bad_vertex_index":
        t = m.tris.copy(); t[3, 1] = 10 ** 6; over["tris"] = t
    elif case == "bad_material_index":
        t = m.tri_mat.copy(); t[0] = 7; over["tm"] = t
    elif case == "bad_node_index":
        t = m.tri_node.copy(); t[0] = 3; over["tn"] = t
    elif case == "rho_sum_above_one":
        over["mats"] = np.array([[0.7, 0.4], [0.1, 0.1]])
    elif case == "negative_rho":
        over["mats"] = np.array([[-0.1, 0.4], [0.1, 0.1]])
    elif case == "root_with_parent":
        p = m.parent.copy(); p[0] = 1; over["parent"] = p
    elif case == "parent_not_before_child":
        p = m.parent.copy(); p[1] = 2; over["parent"] = p
    elif case == "too_many_axes":
        n = m.n_axes.copy(); n[1] = 4; over["n_axes"] = n
    elif case == "nan_vertex":
        v = m.verts.copy(); v[2, 0] = np.nan; over["verts"] = v
    elif case == "zero_axis":
        a = m.axes.copy(); a[1, 0] = 0; over["axes"] = a
    elif case == "inverted_interval":
        lo = m.lo.copy(); lo[1, 0] = 2.0; over["lo"] = lo
    rc, msg, h = _build(lib, m, **over)
    assert rc == -1 and msg and not h.value, (rc, msg)


def test_null_arguments_rejected(lib):
    from paper_2608_07307_amd import _lib as L
    r = L.srp_result()
    p = L.srp_eval_params()
    assert lib.srp_eval(None, C.byref(p), C.byref(r), None, None) == -1
    assert lib.srp_eval_grad(None, C.byref(p), C.byref(r), None, None, None, None) == -1
    assert lib.srp_set_panel_angles(None, None, 0) == -1
    assert lib.srp_set_materials(None, None, 0) == -1
    assert lib.srp_destroy_scene(None) == 0
    assert lib.srp_eval_batch(None, 3, None, None) == -1
    assert lib.srp_eval_grad_batch(None, 2, None, None, 0, None) == -1
    assert lib.srp_profile_read(None, None) == -1
    assert lib.srp_profile_read_launch(None, None) == -1
    assert "null" in lib.srp_last_error().decode()
