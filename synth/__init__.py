"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds input generation only (voxel geometries and random vectors).
It contains none of the solver's arithmetic, so that the oracle and the GPU path
can both be fed from it without sharing any of the method.
"""

from .geometry import (  # noqa: F401
    spheres,
    grf,
    slits,
    porosity,
    random_face_field,
    random_cell_field,
)
