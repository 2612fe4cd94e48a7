"""Pins of the oracle's two-hole configuration interaction (CPU only).

The Slater-Condon matrix is checked against the two-particle Hamiltonian built
independently in the full product space and projected onto antisymmetric
states; the Coulomb integrals against the properties of the device's Green's
function (reciprocity, conjugation, positive semi-definiteness, charge of each
pair density); and the whole construction against closed forms (no
interaction: sums of orbital energies and J = the orbital gap; one orbital:
2 E_0 + (00|00)).
"""

import numpy as np

from oracle import (SI_MATERIAL, Grid, ci_hamiltonian, coulomb_integrals, determinants, exchange,
                    h0_orbital, pair_densities, pair_potentials, poisson_solve, restrict,
                    single_particle)
from oracle.ci import two_body
from synth import sp_device


def _random_integrals(M, rng):
    C = rng.normal(size=(M,) * 4) + 1j * rng.normal(size=(M,) * 4)
    C = C + C.transpose(2, 3, 0, 1)                     # (ik|jl) = (jl|ik)
    C = C + C.transpose(1, 0, 3, 2).conj()              # (ik|jl) = conj((ki|lj))
    return C


def _random_hermitian(n, rng):
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return A + A.conj().T


def test_slater_condon_equals_antisymmetrised_product_space():
    rng = np.random.default_rng(1)
    M = 3
    n = 2 * M
    hsp = _random_hermitian(n, rng)
    C = _random_integrals(M, rng)
    H = ci_hamiltonian(hsp, C)
    assert np.abs(H - H.conj().T).max() < 1e-12
    # product basis chi_u(1) chi_v(2), index u n + v
    H2 = np.zeros((n * n, n * n), dtype=complex)
    for u in range(n):
        for v in range(n):
            for w in range(n):
                for x in range(n):
                    H2[u * n + v, w * n + x] = (hsp[u, w] * (v == x) + (u == w) * hsp[v, x]
                                                + two_body(C, u, v, w, x))
    P = np.zeros((n * n, n * n))
    for u in range(n):
        for v in range(n):
            P[u * n + v, v * n + u] = 1.0
    A = 0.5 * (np.eye(n * n) - P)                       # antisymmetriser (a projector)
    w, U = np.linalg.eigh(A)
    Q = U[:, w > 0.5]                                   # orthonormal antisymmetric basis
    ev_product = np.linalg.eigvalsh(Q.conj().T @ H2 @ Q)
    assert len(ev_product) == len(determinants(M))
    assert np.abs(np.linalg.eigvalsh(H) - ev_product).max() < 1e-10


def test_closed_forms_without_interaction_and_for_one_orbital():
    E = np.array([0.010, 0.013, 0.020])
    M = len(E)
    hsp = np.kron(np.diag(E), np.eye(2))
    ev = np.linalg.eigvalsh(ci_hamiltonian(hsp, np.zeros((M,) * 4)))
    expect = sorted(E[a >> 1] + E[b >> 1] for a, b in determinants(M))
    assert np.abs(ev - expect).max() < 1e-15
    assert abs(exchange(ev) - (E[1] - E[0])) < 1e-15
    C = np.full((1, 1, 1, 1), 0.0123 + 0j)
    ev1 = np.linalg.eigvalsh(ci_hamiltonian(np.kron(np.diag([0.01]), np.eye(2)), C))
    assert ev1.shape == (1,) and abs(ev1[0] - (0.02 + 0.0123)) < 1e-15


def _device_orbitals(M=3):
    d = sp_device("sp_tiny")
    g = Grid(*d.shape, d.h)
    phi0 = poisson_solve(d.pshape, d.h, d.eps_r, d.dirichlet, d.phi_fixed, np.zeros(d.pshape))
    V = d.V_off + restrict(phi0, d.shape, d.offset)
    E, phi = np.linalg.eigh(h0_orbital(g, SI_MATERIAL, V=V).toarray())
    return d, E[:M], phi[:, :M]


def test_coulomb_integrals_are_a_greens_function():
    """Pair densities carry the orbitals' overlaps as charge; the integrals obey
    reciprocity and conjugation, and over pair indices form a Hermitian positive
    semi-definite matrix (the grounded device's Green's function is)."""
    d, E, phi = _device_orbitals(3)
    # a complex orbital basis: a unitary mix of the real eigenvectors
    rng = np.random.default_rng(2)
    Qm, _ = np.linalg.qr(rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
    phi = phi @ Qm
    M = 3
    rho = pair_densities(phi, d.shape, d.h)
    charge = rho.reshape(M, M, -1).sum(axis=2) * d.h ** 3
    assert np.abs(charge - np.eye(M)).max() < 1e-12
    V = pair_potentials(rho, d.pshape, d.offset, d.h, d.eps_r, d.dirichlet)
    C = coulomb_integrals(rho, V, d.shape, d.offset, d.h)
    assert np.abs(C - C.transpose(2, 3, 0, 1)).max() < 1e-12 * np.abs(C).max()
    assert np.abs(C - C.transpose(1, 0, 3, 2).conj()).max() < 1e-12 * np.abs(C).max()
    Q = C.transpose(1, 0, 2, 3).reshape(M * M, M * M)    # Q[(i,k),(j,l)] = (ki|jl)
    assert np.abs(Q - Q.conj().T).max() < 1e-12 * np.abs(Q).max()
    assert np.linalg.eigvalsh(Q).min() > -1e-12 * np.abs(Q).max()
    for i in range(M):
        assert C[i, i, i, i].real > 0 and abs(C[i, i, i, i].imag) < 1e-15


def test_ci_spectrum_is_basis_invariant():
    """The two-hole spectrum depends only on the orbital space, not on the basis
    chosen in it (integrals and single-particle matrix transformed together), and
    the ground state lies below the triplet-like three above it (J > 0)."""
    d, E, phi = _device_orbitals(3)
    M = 3
    rho = pair_densities(phi, d.shape, d.h)
    V = pair_potentials(rho, d.pshape, d.offset, d.h, d.eps_r, d.dirichlet)
    C = coulomb_integrals(rho, V, d.shape, d.offset, d.h)
    hsp = single_particle(E, phi, SI_MATERIAL["delta_so"])
    ev = np.linalg.eigvalsh(ci_hamiltonian(hsp, C))
    rng = np.random.default_rng(3)
    Qm, _ = np.linalg.qr(rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M)))
    phi2 = phi @ Qm
    rho2 = pair_densities(phi2, d.shape, d.h)
    V2 = pair_potentials(rho2, d.pshape, d.offset, d.h, d.eps_r, d.dirichlet)
    C2 = coulomb_integrals(rho2, V2, d.shape, d.offset, d.h)
    from oracle import soi_matrix
    hsp2 = np.kron(Qm.conj().T @ np.diag(E) @ Qm, np.eye(2)) + soi_matrix(phi2,
                                                                         SI_MATERIAL["delta_so"])
    ev2 = np.linalg.eigvalsh(ci_hamiltonian(hsp2, C2))
    assert np.abs(ev - ev2).max() < 1e-10
    assert exchange(ev) > 0
