"""CPU oracle for the hole k.p eigenproblem -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct reference for what the GPU
library computes: the lowest eigenpairs of the finite-difference 6x6
Luttinger-Kohn Hamiltonian with Bir-Pikus strain, Zeeman and Peierls terms and
an electrostatic potential (paper Sec. II.B, Eqs. HNI and LK).  It assembles H
with scipy.sparse from the textbook definitions and diagonalises it with
library routines (dense LAPACK for small grids, ARPACK for large ones).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the GPU path, and the GPU path never
imports it.

Pinning status (see tests/test_oracle_pins.py):
  * kinetic operator          -- pinned (closed-form bulk dispersion along
                                 [001] and [111], hard-wall chain, separable limit)
  * |J m_j> vs |L S> forms     -- pinned (two independent assemblies agree via U)
  * spin-orbit + Zeeman onsite -- pinned (closed-form m_j sectors, Wigner-Eckart)
  * strain                     -- pinned (uniaxial / [111]-shear closed forms,
                                 both assemblies agree)
  * Peierls phases             -- pinned (gauge invariance, time reversal,
                                 Kramers degeneracy at B=0)
  * harmonic confinement       -- pinned (Richardson-extrapolated oscillator levels)
  * Hellmann-Feynman gradient  -- pinned (central finite differences)
  * Zeeman term -- its absolute g-factors are pinned by closed forms at one grid
    point (heavy-hole doublet g = 6 kappa, split-off doublet 4 kappa - 2: the
    Lande factors of 2 kappa mu_B B.J; tests/test_oracle_gmatrix.py); its form and
    sign convention are a reading (the paper prints no Zeeman term).
  * g-matrices and the two-spin model (gmatrix.py) -- pinned (closed-form heavy-hole
    and split-off g at one grid point, Zeeman splitting of the full H(B), gauge-origin
    and basis invariance, mirror-image dots, the paper's t = Delta / sqrt(2) example,
    closed forms of the effective Hamiltonian and of J_perp, J_par)
"""

from .constants import E0, MU_B, E_OVER_HBAR, SI_MATERIAL  # noqa: F401
from .grid import Grid  # noqa: F401
from .hamiltonian import (  # noqa: F401
    hamiltonian_ls, hamiltonian_j, onsite_so_zeeman_ls, strain_orbital_ls,
    U_J_FROM_LS, to_j_basis,
)
from .solve import (  # noqa: F401
    lowest_dense, lowest_arpack, residuals, hf_gradient, gate_potential,
    solve_lowest,
)
from .poisson import (  # noqa: F401
    E_OVER_EPS0, KB, link_permittivity, poisson_operator, poisson_solve, occupancy,
    hole_density, embed, restrict, sp_loop,
)
from .spinfree import h0_orbital, soi_matrix, single_particle  # noqa: F401
from .ci import (  # noqa: F401
    pair_densities, pair_potentials, coulomb_integrals, determinants, ci_hamiltonian, exchange,
)
from .gmatrix import (  # noqa: F401
    field_derivative, g_matrix, symmetric_g, localise, double_dot_g, tunnel_coupling,
    u_minus_eps, rotation, zeeman_fields, effective_hamiltonian, qubit_frame,
    anisotropic_exchange, two_spin_model,
)
