"""FP64 CPU oracle for ray-traced SRP — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never depends on it.

`oracle.c` is the method written out plainly in FP64 (see its header for the
paper passages it follows and the readings of silent points); this module
is a ctypes wrapper around it plus the fixed-visibility finite-difference
gradient and an FP64 reference propagator.
"""
from .core import (  # noqa: F401
    build,
    eval_srp,
    grid_of,
    articulate,
    node_transforms,
    shade_frozen,
    fd_gradients,
    OracleResult,
    threads,
    diffuse_set,
    record_slots,
    shade_frozen_dir,
    fd_dir_jacobian,
)
