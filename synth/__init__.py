"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds problem descriptions (grid sizes, spacing, time step, face
masks), seeded media (permittivity / conductivity on the FEM node lattice),
source parameters and seeded noise.  It holds none of the solver's arithmetic:
no operators, no time stepping, no source time functions.
"""

from .configs import (  # noqa: F401
    FACE_TOP, FACE_BOTTOM, FACE_XMIN, FACE_XMAX, FACE_YMIN, FACE_YMAX, FACE_ALL,
    SRC_SINE1, SRC_GAUSS_SINE, SRC_DIPOLE,
    ProblemDesc, Source, Workload,
    fem_layers, fem_node_coords,
    c1, c2, c3, probe288, stream224, small, batch_mix, noise, initial_pulses, with_steps, gauss_sine, oblique_wave,
    plane_wave_switch, Request, serving_requests, meshref_marks, refined_mesh, refined_values, aligned_box,
)
