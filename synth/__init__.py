"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package holds node sets, normals and initial conditions only.  It holds
none of the RBF-FD arithmetic: neither the HIP path nor the CPU oracle lives
here, and both consume what it produces.
"""
from .nodes import (  # noqa: F401
    fibonacci_sphere,
    jittered_torus,
    torus_grid_for_count,
    ellipsoid,
    blob,
    planar_patch,
    surface_batch,
    icosahedral_sphere,
    staggered_torus,
    torus_angles,
    cached,
)
from .fields import (  # noqa: F401
    real_sph_harm,
    random_sph_harm_ic,
    schnakenberg_ic,
    sphere_heat_series,
    bump_centres,
    sphere_forced,
    torus_forced,
)
