"""Plain CPU FP64 oracle for the matrix-free SIMP hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports it, and it never
imports the product path: the two share no code.  Only the seeded problem
generators in ``synth`` serve both.

Everything here is written for clarity, not speed: NumPy/SciPy in FP64,
no blocking, no fusion, each function citing the passage of the paper
(arXiv 2204.06204, "First-Order Bilevel Topology Optimization for Fast
Mechanical Design") that it follows.  The paper is two-dimensional and
never fixes an element; here it is lifted to 3D hex8 elements, and each
function's docstring states the reading it takes of an unstated detail.

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: Gauss quadrature and rigid-body modes for KE, the patch test and a
cantilever beam for the operator, SciPy CG for the inner solver, brute
force for the filter and the projection, finite differences for the
gradient.
"""
from .element import material_lame, element_stiffness, KE_DIAG
from .grid import Grid
from .operator import simp_scale, simp_dscale, assemble_K, apply_K, apply_K_rows, jacobi_diag
from .solve import solve_direct, pcg_ref, pcg_to_tol, krylov_step_ref
from .sensitivity import (element_energy, element_bilinear, element_bilinear_at, compliance_gradient,
                          adjoint_gradient)
from .density_filter import (cone_filter_matrix, filter_forward, filter_transpose, filter_weight_sums_at,
                             filter_forward_at, filter_transpose_at)
from .projection import project_volume_ref, project_bisect, box_clamp
from .outer import outer_step_ref, run_outer_ref, step_size, true_objective, relative_projection_error

__all__ = [
    "material_lame", "element_stiffness", "KE_DIAG", "Grid",
    "simp_scale", "simp_dscale", "assemble_K", "apply_K", "apply_K_rows", "jacobi_diag",
    "solve_direct", "pcg_ref", "pcg_to_tol", "krylov_step_ref",
    "element_energy", "element_bilinear", "element_bilinear_at", "compliance_gradient", "adjoint_gradient",
    "cone_filter_matrix", "filter_forward", "filter_transpose", "filter_weight_sums_at", "filter_forward_at",
    "filter_transpose_at",
    "project_volume_ref", "project_bisect", "box_clamp",
    "outer_step_ref", "run_outer_ref", "step_size", "true_objective", "relative_projection_error",
]
