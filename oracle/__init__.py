"""Plain, slow, FP64 CPU oracle for the cell-centred multigrid solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  The GPU library
never routes through it and shares no code with it: the two meet only in the
seeded input generators of ``workloads``, which hold none of the method's
arithmetic.

What it computes follows the AMReX paper (Zhang et al., "AMReX:
Block-Structured Adaptive Mesh Refinement for Multiphysics Applications"):

* index-space boxes, box arrays and ghost cells ("Basic data structures",
  "Containers for mesh data", "Operations on a level");
* the ghost-cell exchange between boxes of one level, written as a brute-force
  intersection of every grown box with every (periodically shifted) box
  ("Operations on a level", "Communication");
* the variable-coefficient cell-centred operator of the "Linear Solvers"
  section, written here as ``alpha*a*phi - beta*div(b grad phi) = f`` with
  scalar alpha/beta, ``a`` per cell and ``b`` per face;
* a geometric multigrid V-cycle with a CG bottom solve ("Linear Solvers"),
  with averaging restriction and piecewise-constant interpolation ("Operations
  between levels");
* the nodal solver of the same section (``oracle.nodal``): the trilinear
  finite-element operator of -div(sigma grad phi) built from the cells' moment
  integrals, Galerkin coarse operators, Jacobi smoothing, CG bottom.

The paper does not fix the smoother, the transfer operators, the coefficient
coarsening, the boundary stencil, the bottom tolerance or the stopping norm;
each function states which reading it takes.  Every array is float64 unless a
function says otherwise.
"""

from .boxes import (  # noqa: F401
    Box,
    box_shape,
    grow,
    intersect,
    coarsen_box,
    refine_box,
    validate_boxarray,
    mg_hierarchy,
    copy_tags,
    fill_boundary,
)
from .mlmg import (  # noqa: F401
    Level,
    make_level,
    coarsen_level,
    new_cell_data,
    stencil,
    apply_op,
    residual,
    gsrb_halfsweep,
    restrict,
    prolong_add,
    cg_bottom,
    bicgstab_bottom,
    vcycle,
    solve,
    solve_refine,
    pcg_solve,
    vcycle_precond,
    max_norm,
    Opts,
    build_levels,
    cast_level,
    colour_mask,
    valid,
    is_singular,
)
from .adjoint import grad_logb, loss, gather_cells, gather_faces  # noqa: F401
