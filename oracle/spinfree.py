"""Spin-free single-particle basis and its spin-orbit matrix -- TEST INFRASTRUCTURE
ONLY (tests, smoke check, CPU baseline).

The paper builds the basis of its configuration-interaction step from the
eigenstates of H_0 = H_DKK + V_DQD + H'_PB (Eq. H0): the Hamiltonian without the
spin-orbit term, at zero magnetic field.  In the |L S> basis H_0 is then two
identical 3 x 3 orbital blocks, one per spin, and only one of them is
diagonalised (Sec. II.D).  Spin-orbit coupling returns as matrix elements
between the spin-orbitals phi_i (x) s (Eq. H1; Fig. 2d-e).

  h0_orbital    the 3N x 3N real symmetric orbital block: the spin-up block of
                the |L S> Hamiltonian assembled with delta_so = 0 and B = 0
  soi_matrix    <phi_i s| H_SO |phi_j s'>, H_SO = (Delta_0 / 3)(1 - sum_a sigma_a (x) L_a)
                on every grid point, index 2 i + s (s = 0 up, 1 down)
  single_particle  diag(E_i) (x) 1_2 + the spin-orbit matrix: the single-particle
                part of the configuration-interaction Hamiltonian in this basis

Orbital vectors are (3N, M) arrays with index 3 p + b (b = X, Y, Z), the layout of
the library's spin-free output.
"""

import numpy as np

from .constants import SI_MATERIAL
from .hamiltonian import hamiltonian_ls, onsite_so_zeeman_ls


def h0_orbital(grid, material=SI_MATERIAL, V=None, strain=None):
    """The orbital (spin-up) block of H without spin-orbit coupling, at B = 0."""
    mat = dict(material)
    mat["delta_so"] = 0.0
    H = hamiltonian_ls(grid, mat, V=V, strain=strain, B=(0.0, 0.0, 0.0)).tocsr()
    N = grid.npts
    up = (6 * np.arange(N)[:, None] + np.arange(3)[None, :]).ravel()   # 6 p + b -> 3 p + b
    h = H[up][:, up]
    if abs(h.imag).max() > 0:
        raise AssertionError("the spin-free block at B = 0 must be real")
    return h.real.tocsr()


def soi_matrix(phi, delta_so):
    """2M x 2M spin-orbit matrix of the spin-orbitals phi_i (x) s, index 2 i + s."""
    phi = np.asarray(phi)
    M = phi.shape[1]
    p = phi.reshape(-1, 3, M)                                   # (N, b, i)
    O = np.einsum("pbi,pcj->ibjc", p.conj(), p)                # <phi_i,b | phi_j,c>
    mat = dict(SI_MATERIAL)
    mat["delta_so"] = float(delta_so)
    hso = onsite_so_zeeman_ls(mat).reshape(2, 3, 2, 3)         # [s, b, s', c], spin-major
    out = np.einsum("ibjc,sbtc->isjt", O, hso)
    return out.reshape(2 * M, 2 * M)


def single_particle(E, phi, delta_so):
    """diag(E_i) (x) 1_2 + the spin-orbit matrix."""
    E = np.asarray(E, dtype=float)
    return np.kron(np.diag(E), np.eye(2)) + soi_matrix(phi, delta_so)
