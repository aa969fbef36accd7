"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This package only *generates* inputs: spacecraft meshes with their kinematic
trees and optical coefficients, sun-direction sets and hinge-angle sets.  It
holds none of the SRP method's arithmetic (no articulation, ray grid,
intersection or momentum law); both the oracle and the HIP path consume what
it produces, and neither imports the other.
"""
from .scenes import (  # noqa: F401
    Scene,
    plate,
    stacked_plates,
    hinged_plate,
    cube,
    dihedral,
    icosphere,
    box_wing,
    box_wing_2axis,
    procedural_spacecraft,
    procedural_sized,
    uneven_batch_specs,
    greebled_spacecraft,
    merge_static,
)
from .dirs import random_dirs, fibonacci_dirs  # noqa: F401
from .workloads import c2_batch, c3_spad, c4_uneven, c5_batch, diffuse_batch  # noqa: F401
