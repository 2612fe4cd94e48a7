"""Eigen-solves and derived quantities of the oracle (library primitives only).

The lowest `nev` eigenpairs of the Hermitian H are a plain definition; the
oracle takes them from LAPACK (dense) or ARPACK (the paper's own comparison
system, Sec. II.B).  Eigenvectors are returned in |J m_j> order, normalised to
sum |psi|^2 = 1 over grid and components (no volume factor).
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .hamiltonian import hamiltonian_ls, to_j_basis


def lowest_dense(H, nev):
    """Lowest nev eigenpairs of a (sparse or dense) Hermitian matrix via LAPACK."""
    A = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    w, v = sla.eigh(A, subset_by_index=(0, nev - 1), driver="evr")
    return w, v


def lowest_arpack(H, nev, tol=1e-13, guard=4, ncv=None, v0=None, maxiter=None):
    """Lowest nev eigenpairs via ARPACK (implicitly restarted Lanczos, 'SA')."""
    k = nev + guard
    n = H.shape[0]
    k = min(k, n - 2)
    if ncv is None:
        ncv = min(n - 1, max(2 * k + 1, 64))
    w, v = spla.eigsh(H, k=k, which="SA", tol=tol, ncv=ncv, v0=v0, maxiter=maxiter)
    order = np.argsort(w)
    return w[order][:nev], v[:, order][:, :nev]


def residuals(H, E, psi):
    """r_n = || H psi_n - E_n psi_n ||_2 for unit-norm columns of psi (6N, k)."""
    R = H @ psi - psi * np.asarray(E)[None, :]
    return np.linalg.norm(R, axis=0)


def solve_lowest(grid, material, nev, V=None, strain=None, B=(0.0, 0.0, 0.0),
                 method="auto", tol=1e-13):
    """Lowest nev eigenpairs of H_NI; returns (E, psi_J (6N, nev), H_ls)."""
    H = hamiltonian_ls(grid, material, V=V, strain=strain, B=B)
    if method == "auto":
        method = "dense" if H.shape[0] <= 6000 else "arpack"
    if method == "dense":
        E, v = lowest_dense(H, nev)
    else:
        E, v = lowest_arpack(H, nev, tol=tol)
    return E, to_j_basis(v), H


def gate_potential(V_bg, L, Vg):
    """V(r) = V_bg(r) + sum_g L_g(r) V_g  (linear gate -> potential map)."""
    return np.asarray(V_bg, dtype=float) + np.tensordot(np.asarray(Vg, dtype=float),
                                                        np.asarray(L, dtype=float), axes=1)


def hf_gradient(psi, w, L):
    """Hellmann-Feynman gradient of sum_n w_n E_n with respect to gate voltages.

    dE_n/dV_g = <psi_n| L_g |psi_n> because dH/dV_g = L_g(r) times the identity
    on the six components.  psi: (6N, nev) unit-norm columns (any basis), w: (nev,),
    L: (G, N).  Returns (G,).
    """
    nev = psi.shape[1]
    dens = (np.abs(np.asarray(psi)) ** 2).reshape(-1, 6, nev).sum(axis=1)  # (N, nev)
    return np.asarray(L, dtype=float) @ (dens @ np.asarray(w, dtype=float))
