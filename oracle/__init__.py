"""Oracle for the discrete biharmonic field extension (test infrastructure only).

This package is a plain, slow CPU reference written from the paper
"Extending fields in a level set method by solving a biharmonic equation"
(Moroney, Lusmore, McCue, McElwain). It exists to check the GPU library and
is never part of the product path: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. It shares no code
with the HIP library and imports nothing from the package.

Everything is float64 (residuals for iterative refinement in numpy
``longdouble``); see ``biharmonic.py`` for each function and the passage of
the paper it follows (``biharmonic3d.py`` for three dimensions).
"""
from .biharmonic import (  # noqa: F401
    NEUMANN, PERIODIC, DIRICHLET,
    known_mask, second_difference_1d, laplacian, biharmonic_matrix,
    stencil_padded, stencil_padded_ld, rhs, reduced_system, extend_direct,
    eigenvalues_1d, transform_1d, spectral_preconditioner, pcg,
    true_relative_residual, relative_l2,
)
from .biharmonic3d import (  # noqa: F401
    laplacian_3d, biharmonic_matrix_3d, stencil_padded_3d, rhs_3d, reduced_system_3d,
    extend_direct_3d, spectral_preconditioner_3d, pcg_3d, true_relative_residual_3d,
)
