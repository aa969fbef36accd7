"""Seeded sun-direction sets (unit vectors, body frame, spacecraft -> Sun)."""
from __future__ import annotations

import numpy as np


def random_dirs(seed: int, n: int = 1) -> np.ndarray:
    """n directions uniform on the sphere: normalised standard normals."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def fibonacci_dirs(n: int) -> np.ndarray:
    """Fibonacci sphere: z_i = 1 - (2i+1)/n, phi_i = i * pi * (3 - sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
