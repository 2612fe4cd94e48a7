"""Configuration interaction for two holes -- TEST INFRASTRUCTURE ONLY (tests,
smoke check, CPU baseline).

The paper expands the two-hole states in Slater determinants of spin-orbitals
phi_i (x) s built from the spin-free orbitals (Eq. Phi, Sec. II.D), brings back
spin-orbit coupling through the single-particle matrix and the Coulomb
interaction through two-particle integrals whose potentials come from Poisson
solves of the orbital pair densities (Fig. 2d-e), and diagonalises the
resulting configuration-interaction Hamiltonian (Eq. J and Fig. 2f: the
exchange J as a function of detuning).  Readings taken here:

  * pair density rho_ik(r) = sum_b conj(phi_i,b(r)) phi_k,b(r) / h^3 (one hole
    charge per unit norm), its potential V_ik from the Poisson problem of the
    device with every electrode grounded (the gates' own potential is already in
    the orbitals), complex densities solved as real and imaginary parts;
  * Coulomb integrals (ik|jl) = sum_r h^3 rho_ik(r) V_jl(r) in eV (hole charge e);
  * spin-orbitals u = 2 i + s; <uv|wx> = delta(s_u, s_w) delta(s_v, s_x) (i_u i_w | i_v i_x);
  * determinants |u v>, u < v, in lexicographic order; matrix elements
    <uv|H|wx> = h_uw d_vx + h_vx d_uw - h_ux d_vw - h_vw d_ux + <uv|wx> - <uv|xw>
    (the two-particle Slater-Condon rules), h the single-particle matrix;
  * exchange J = mean of the three states above the ground state minus the
    ground state (the triplet manifold over the singlet at B = 0).
"""

import itertools

import numpy as np

from .poisson import embed, poisson_solve


def pair_densities(phi, shape, h):
    """rho[i, k] = sum_b conj(phi_i,b) phi_k,b / h^3 on the Schroedinger grid, (M, M, *shape)."""
    M = phi.shape[1]
    p = np.asarray(phi).reshape(-1, 3, M)
    rho = np.einsum("pbi,pbk->ikp", p.conj(), p) / h ** 3
    return rho.reshape((M, M) + tuple(shape))


def pair_potentials(rho, pshape, offset, h, eps_r, dirichlet):
    """V[i, k] on the Poisson box for every pair density, electrodes grounded."""
    M = rho.shape[0]
    zero = np.zeros(pshape)
    V = np.zeros((M, M) + tuple(pshape), dtype=complex)
    for i in range(M):
        for k in range(M):
            re = poisson_solve(pshape, h, eps_r, dirichlet, zero, embed(rho[i, k].real, pshape,
                                                                        offset))
            im = poisson_solve(pshape, h, eps_r, dirichlet, zero, embed(rho[i, k].imag, pshape,
                                                                        offset))
            V[i, k] = re + 1j * im
    return V


def coulomb_integrals(rho, V, shape, offset, h):
    """C[i, k, j, l] = (ik|jl) = sum_r h^3 rho_ik(r) V_jl(r) over the Schroedinger grid."""
    ox, oy, oz = offset
    nx, ny, nz = shape
    Vs = V[:, :, ox:ox + nx, oy:oy + ny, oz:oz + nz]
    M = rho.shape[0]
    return h ** 3 * np.einsum("ikp,jlp->ikjl", rho.reshape(M, M, -1), Vs.reshape(M, M, -1))


def determinants(M):
    """Two-hole determinants (u, v), u < v, over the 2M spin-orbitals u = 2 i + s."""
    return list(itertools.combinations(range(2 * M), 2))


def two_body(C, u, v, w, x):
    """<uv|wx> in spin-orbitals from spatial (ik|jl)."""
    if (u & 1) != (w & 1) or (v & 1) != (x & 1):
        return 0.0
    return C[u >> 1, w >> 1, v >> 1, x >> 1]


def ci_hamiltonian(hsp, C):
    """K x K configuration-interaction matrix over determinants (u < v)."""
    M = hsp.shape[0] // 2
    dets = determinants(M)
    K = len(dets)
    H = np.zeros((K, K), dtype=complex)
    d = np.eye(2 * M)
    for a, (u, v) in enumerate(dets):
        for b, (w, x) in enumerate(dets):
            H[a, b] = (hsp[u, w] * d[v, x] + hsp[v, x] * d[u, w] - hsp[u, x] * d[v, w]
                       - hsp[v, w] * d[u, x] + two_body(C, u, v, w, x) - two_body(C, u, v, x, w))
    return H


def exchange(E):
    """J = mean(E_1, E_2, E_3) - E_0 from the ascending two-hole spectrum."""
    E = np.sort(np.asarray(E, dtype=float))
    return float(E[1:4].mean() - E[0])
