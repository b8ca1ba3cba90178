"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package builds surfaces, quadrature nodes, weights, normals, QBX centers and
densities.  It holds none of the layer-potential or FMM arithmetic: it only produces the
arrays that both sides consume.
"""

from .geometry import (  # noqa: F401
    Workload,
    add_point_targets,
    fresh_densities,
    icosphere,
    make_workload,
    oversampled_workload,
    workload_c1,
    workload_c2,
    workload_c3,
    c3_surface_params,
    workload_c4,
    workload_tiny,
)
