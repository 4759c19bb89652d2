"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package produces *data only*: voxel masks and plain scalar case
parameters (lattice sizes, relaxation time, inlet amplitude, seeds).  It holds
none of the lattice Boltzmann arithmetic, so the CPU oracle and the HIP library
can both consume its output without sharing any of the method's code.

The geometries stand in for the paper's vessel and aneurysm models (the
idealized sidewall aneurysm of Sec. 2.2.2 and the patient-specific case of
Sec. 2.2.3), whose CAD and segmentation data are not available.
"""

from .geometry import (  # noqa: F401
    SOLID, FLUID, INLET, OUTLET,
    PERIODIC_X, PERIODIC_Y, PERIODIC_Z,
    Case, pipe_case, aneurysm_case, batch_cases, fluid_count,
    random_tiny_case, periodic_box_case, channel_case, open_pipe_case,
)
from .walls import wall_links, fluid_predicate, wall_distances, random_wall_distances  # noqa: F401
