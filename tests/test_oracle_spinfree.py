"""Pins of the oracle's spin-free basis and spin-orbit matrix (CPU only).

The checks compare against what fixes them independently: the structure of H
without spin-orbit coupling at B = 0 (two identical, uncoupled spin blocks), the
exact spectrum of the full Hamiltonian when the spin-orbital basis is complete,
the closed-form Gamma8 / Gamma7 splitting of a single grid point, and the trace
and Kramers structure of the spin-orbit matrix.
"""

import numpy as np

from oracle import SI_MATERIAL, Grid, hamiltonian_ls, h0_orbital, single_particle, soi_matrix
from oracle.constants import E0


def _fields(grid, seed):
    rng = np.random.default_rng(seed)
    V = rng.normal(0.0, 0.05, grid.npts)
    strain = rng.normal(0.0, 2e-3, (grid.npts, 6))
    return V, strain


def test_spin_free_h_is_two_identical_uncoupled_blocks():
    g = Grid(4, 3, 3, 0.5)
    V, strain = _fields(g, 1)
    mat = dict(SI_MATERIAL)
    mat["delta_so"] = 0.0
    H = hamiltonian_ls(g, mat, V=V, strain=strain).toarray().reshape(g.npts, 6, g.npts, 6)
    h0 = h0_orbital(g, SI_MATERIAL, V=V, strain=strain).toarray().reshape(g.npts, 3, g.npts, 3)
    assert np.abs(h0 - h0.transpose(2, 3, 0, 1)).max() < 1e-13       # real symmetric
    assert np.abs(H[:, :3, :, :3] - h0).max() == 0.0
    assert np.abs(H[:, 3:, :, 3:] - h0).max() < 1e-13               # spin down: the same block
    assert np.abs(H[:, :3, :, 3:]).max() == 0.0                      # no spin coupling
    assert np.abs(H[:, 3:, :, :3]).max() == 0.0


def test_complete_basis_reproduces_the_full_spectrum():
    """With all 3N orbitals, diag(E) (x) 1 + SOI is H with spin-orbit coupling
    written in another basis: its eigenvalues are the full Hamiltonian's."""
    g = Grid(3, 3, 2, 0.5)
    V, strain = _fields(g, 2)
    E, phi = np.linalg.eigh(h0_orbital(g, SI_MATERIAL, V=V, strain=strain).toarray())
    h = single_particle(E, phi, SI_MATERIAL["delta_so"])
    assert np.abs(h - h.conj().T).max() < 1e-14
    full = np.linalg.eigvalsh(hamiltonian_ls(g, SI_MATERIAL, V=V, strain=strain).toarray())
    assert np.abs(np.linalg.eigvalsh(h) - full).max() < 1e-11


def test_single_point_gamma8_gamma7():
    """One grid point, no potential or strain: the orbital block is the kinetic
    centre 2 E0 (L + 2M) / h^2 = 6 E0 gamma1 / h^2 on X, Y, Z; with spin-orbit
    coupling the six states split into a Gamma8 quartet there and a Gamma7
    doublet Delta_0 above it."""
    h = 0.5
    g = Grid(1, 1, 1, h)
    c = 6.0 * E0 * SI_MATERIAL["gamma1"] / h ** 2
    h0 = h0_orbital(g, SI_MATERIAL).toarray()
    assert np.abs(h0 - c * np.eye(3)).max() < 1e-12
    E, phi = np.linalg.eigh(h0)
    ev = np.linalg.eigvalsh(single_particle(E, phi, SI_MATERIAL["delta_so"]))
    d = SI_MATERIAL["delta_so"]
    assert np.abs(ev - np.array([c] * 4 + [c + d] * 2)).max() < 1e-12


def test_soi_matrix_trace_hermiticity_and_kramers():
    """For M orthonormal orbitals the spin-orbit matrix is Hermitian with trace
    2 M Delta_0 / 3 (sigma_a is traceless), and diag(E) (x) 1 + SOI has doubly
    degenerate eigenvalues (time reversal at B = 0)."""
    g = Grid(5, 3, 3, 0.5)
    V, strain = _fields(g, 3)
    E, phi = np.linalg.eigh(h0_orbital(g, SI_MATERIAL, V=V, strain=strain).toarray())
    M, d = 7, SI_MATERIAL["delta_so"]
    S = soi_matrix(phi[:, :M], d)
    assert np.abs(S - S.conj().T).max() < 1e-15
    assert abs(np.trace(S).real - 2 * M * d / 3) < 1e-14 and abs(np.trace(S).imag) < 1e-15
    ev = np.linalg.eigvalsh(single_particle(E[:M], phi[:, :M], d))
    assert np.abs(ev[0::2] - ev[1::2]).max() < 1e-12
    # a unitary change of basis inside the orbital space leaves the spectrum unchanged
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M)))
    h1 = soi_matrix(phi[:, :M] @ Q, d) + np.kron(Q.conj().T @ np.diag(E[:M]) @ Q, np.eye(2))
    assert np.abs(np.linalg.eigvalsh(h1) - ev).max() < 1e-12
