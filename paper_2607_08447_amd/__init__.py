"""MI355X-native solver for the lowest hole eigenpairs of the finite-difference
6x6 Luttinger-Kohn k.p Hamiltonian (Bir-Pikus strain, Zeeman and Peierls
terms, gate potential), the Schroedinger step of the self-consistent
Schroedinger-Poisson loop of arXiv 2607.08447.

The computation runs in hand-written HIP kernels for gfx950 behind the C ABI in
include/hkp.h; this package is its Python binding.  Importing it loads the
in-tree libhkp.so and fails if it is missing.
"""

from ._lib import HkpError, lib  # noqa: F401
from .api import (  # noqa: F401
    SI, EigvalsFromPotential, SolveResult, apply, autotune, autotune_block, filter_step,
    filter_step2, gate_potential,
    hf_grad, solve, solve_batch, solve_sweep, workspace_bytes, poisson, occupancy, hole_density,
    sp_solve, SPResult, soi_matrix, ci_solve, CIResult, g_matrices, GMatrixResult, two_spin_model,
    poisson_preconditioner, tuned_shape, tune_cache_save, tune_cache_load, tune_cache_clear,
)

__version__ = "1.0.0"
