"""CPU oracle for the Wilson-Dirac operator -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 numpy code that states what the GPU library computes. Only
the tests, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path (the HIP library and its Python binding) never does, and
this package imports nothing from the product path. The two sides share only
the seeded input generator in ``lattice_inputs``.

Every function here is pinned by tests that do not re-type its formulas:
closed forms of the free field, gamma5-hermiticity, gauge covariance,
translation covariance, the relation to eq. (1) of the paper, and a dense
matrix built entry by entry on tiny lattices; the solvers of D x = b (plain
and even-odd preconditioned) against dense solves and dense block
elimination of that matrix.
"""

from .wilson_ref import (  # noqa: F401
    GAMMA, GAMMA5, gamma5_apply, shift, dslash, dslash_dagger, dslash_multi, hopping_paper,
    dslash_sites, dense_matrix, site_index, site_coords, flops_per_site,
)
from .cg_ref import cg_normal, normal_op  # noqa: F401
from .solve_ref import (  # noqa: F401
    parity, restrict, hopping, hopping_dagger, schur_odd, schur_odd_dagger, eo_source,
    eo_reconstruct, cg_hpd, wilson_residual, solve_wilson, solve_wilson_eo, gamma5_schur,
)
