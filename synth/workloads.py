"""The benchmark workloads as seeded arrays (meshes, Sun directions, hinge
angles); shared by the benchmark and the full-size tests.  No SRP arithmetic.

  c2_batch   ~50k-triangle procedural spacecraft (seed 2), a batch of E
             attitudes: Fibonacci Sun directions, the two wing-root hinges
             drawn U(-90, 90) deg (seed 1002), other joints at 0; 1024^2, B = 2.
  c3_spad    the same mesh, 4096 Fibonacci directions x 8 root-hinge angles
             linspace(-90, 90) deg on both roots (direction-major), 512^2, B = 1.
  c4_uneven  64 procedural scenes of 1k..500k triangles, grids 256..2048, root
             hinges U(-90, 90) deg, random Sun directions (seed 4), B = 1.
  c5_batch   ~1M-triangle greebled spacecraft (seed 5), 256 Fibonacci
             directions, all 64 hinges U(-0.3, 0.3) rad (seed 1005), 2048^2, B = 1.
  diffuse_batch  the c2 mesh and attitudes at the paper's ray-traced setting
             (256^2 window, two secondary levels, 16 diffuse rays per hit).
"""
from __future__ import annotations

import numpy as np

from .dirs import fibonacci_dirs
from .scenes import greebled_spacecraft, procedural_sized, procedural_spacecraft, uneven_batch_specs

HALF_PI = np.pi / 2


def c2_batch(E: int = 64):
    mesh = procedural_spacecraft(seed=2)
    dirs = fibonacci_dirs(E)
    rng = np.random.default_rng(1002)
    angles = np.zeros((E, mesh.n_dof))
    angles[:, [0, mesh.n_dof // 2]] = rng.uniform(-HALF_PI, HALF_PI, size=(E, 2))
    return mesh, dirs, angles, 1024, 2


def c3_spad(n_dirs: int = 4096, n_angles: int = 8):
    mesh = procedural_spacecraft(seed=2)
    d = fibonacci_dirs(n_dirs)
    a = np.linspace(-HALF_PI, HALF_PI, n_angles)
    dirs = np.repeat(d, n_angles, axis=0)
    angles = np.zeros((n_dirs * n_angles, mesh.n_dof))
    angles[:, 0] = np.tile(a, n_dirs)
    angles[:, mesh.n_dof // 2] = np.tile(a, n_dirs)
    return mesh, dirs, angles, 512, 1


def c4_uneven(n: int = 64):
    """Returns a list of (mesh, angles, sun_dir, N) and B."""
    out = []
    for s in uneven_batch_specs(seed=4, n=n):
        m = procedural_sized(s["seed"], s["target_tris"])
        ang = np.zeros(m.n_dof)
        ang[0], ang[m.n_dof // 2] = s["root_angles"]
        out.append((m, ang, s["sun_dir"], s["n"]))
    return out, 1


def c5_batch(E: int = 256):
    mesh = greebled_spacecraft(seed=5)
    dirs = fibonacci_dirs(E)
    rng = np.random.default_rng(1005)
    angles = rng.uniform(-0.3, 0.3, size=(E, mesh.n_dof))
    return mesh, dirs, angles, 2048, 1


def diffuse_batch(E: int = 64):
    """Returns mesh, dirs, angles, N, B and K (diffuse rays per emitting hit)."""
    mesh, dirs, angles, _, _ = c2_batch(E)
    return mesh, dirs, angles, 256, 2, 16
