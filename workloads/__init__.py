"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This package holds no arithmetic of the DoGIP method: it only produces the
problem data (simplex meshes of the unit square/cube, per-element coefficients,
right-hand sides and trial vectors) with the shapes and value distributions of
the paper's experiments (Section 3, mesh family M_N with 2N^2 triangles or 6N^3
tetrahedra) and of the benchmark workloads built on them.
"""

from .generate import (  # noqa: F401
    unit_mesh,
    cell_centroids,
    coef_uniform,
    coef_aniso_2d,
    coef_aniso_3d,
    gaussian_field_rff,
    coef_lognormal,
    theta_normal,
    random_vector,
    batch_spec,
    WORKLOADS,
    rng_for,
)
