"""Seeded synthetic inputs for the material-weighted Laplacian -div(sigma grad u) = f.

This package only builds problems: structured Q1 meshes, element material tensors,
the assembled stiffness matrix and load vector, and the serving request stream.
It holds none of the multigrid method's arithmetic; the CPU oracle and the HIP
library both consume the arrays it returns.
"""

from .q1 import (  # noqa: F401
    Problem,
    box_mesh,
    assemble_q1,
    config1_checkerboard_2d,
    layered_stack_3d,
    rotated_anisotropic_3d,
    two_domain_2d,
    poisson_box,
    structured_hex_nodes,
    assemble_hex,
    annulus_3d,
    serving_stream,
    problem_from_request,
    ulp_perturbed,
    seeded_start,
    problem_digest,
)
