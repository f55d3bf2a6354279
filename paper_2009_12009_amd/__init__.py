"""MI355X-native block-structured multigrid (the MLMG solve of AMReX-style AMR).

The compute path is libamrmg.so (hand-written gfx950 HIP kernels behind a C
ABI, include/amrmg.h).  Importing the package loads that library and raises
ImportError if it is missing: there is no CPU fallback.
"""

from . import _lib  # noqa: F401  (loads libamrmg.so)
from ._lib import MGError  # noqa: F401
from .multifab import MultiFab, global_to_xfast, xfast_to_global  # noqa: F401
from .solver import (  # noqa: F401
    MLMG,
    CompositeMLMG,
    copy_tags,
    fill_boundary,
    fill_boundary_noalloc,
    num_levels,
    release_caches,
    stream_copy,
    workspace_bytes,
)
from .autograd import MGSolve, mg_solve  # noqa: F401
from .nodal import NodalMLMG, nodal_workspace_bytes  # noqa: F401
