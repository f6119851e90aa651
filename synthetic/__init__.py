"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws numbers: vertex coordinates and cell vertex ids of
box and general hexahedral meshes, nodal displacement vectors and random test
vectors.  It holds none of the finite
element arithmetic (no basis functions, no geometry map, no material law), so
that the oracle and the HIP path can both be fed from it without sharing any
of the method's code.
"""

from .configs import CONFIGS, Workload, get_config
from .generators import (
    box_vertices,
    box_counts,
    sine_displacement,
    random_vectors,
    rng_for,
    clamp_and_twist,
)
from .hexmesh import box_cells, cube_in_cube, cube_rotations, relabel, sine_field

__all__ = [
    "CONFIGS",
    "Workload",
    "get_config",
    "box_vertices",
    "box_counts",
    "sine_displacement",
    "random_vectors",
    "rng_for",
    "clamp_and_twist",
    "box_cells",
    "cube_in_cube",
    "cube_rotations",
    "relabel",
    "sine_field",
]
