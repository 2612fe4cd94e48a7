"""Electrostatics and the self-consistent Schroedinger-Poisson loop of the
oracle -- TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

The paper closes its Schroedinger solve in a self-consistent loop (Sec. II.B,
Fig. 2a): the hole eigenstates give a hole density, a 3-D finite-difference
Poisson equation with the gate electrodes as fixed-potential (Dirichlet) nodes
and zero normal field on every other outer face gives the electrostatic
potential, and the potential goes back into the Hamiltonian until nothing
changes.  The paper fixes neither the discretisation nor the occupancy rule nor
the update; the readings taken here are:

  * Poisson domain: a box of P grid points with the spacing h of the
    Schroedinger grid, which sits inside it at an integer offset.
  * -div(eps_r grad phi) = (e/eps0) rho, 7-point finite differences; the
    permittivity of a link between two nodes is the harmonic mean of the
    nodes' values (exact flux continuity for an interface midway between
    them); links leaving the box carry no flux (Neumann); Dirichlet nodes keep
    their given potential.  rho in e/nm^3 (holes positive), phi in V.
  * Hole energy: V(r) = V_off(r) + phi(r) (eV): in the hole picture the
    electron potential energy -e phi enters with the opposite sign.
  * Occupancy: each eigenstate (a spinor) holds at most one hole, Fermi-Dirac
    in the hole energy, f_n = 1 / (1 + exp((E_n - mu) / kT)), with mu fixed by
    sum_n f_n = n_holes over the computed states.
  * Hole density p(r) = sum_n f_n sum_c |psi_n,c(r)|^2 / h^3 (nm^-3), psi
    normalised to sum |psi|^2 = 1 on the grid.
  * Update: Anderson mixing of the potential over the last m iterations (m = 0:
    plain linear mixing).  With the residual F(phi) = phi_out(phi) - phi, the
    next input is phi + a F - (dX + a dF) g, where the columns of dX and dF are
    the differences of successive inputs and residuals and g minimises
    |F - dF g|_2 (Anderson, J. ACM 12, 547 (1965); the "type II" form).  The
    loop stops when max |phi_out - phi_in| <= tol; the potential returned is the
    last phi_in, the one the returned eigenpairs belong to.

Everything is plain numpy / scipy in float64; the Poisson system is solved
directly (sparse LU).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .constants import SI_MATERIAL
from .grid import Grid
from .solve import solve_lowest

# e / eps0 in V nm (e = 1.602176634e-19 C, eps0 = 8.8541878128e-12 F/m)
E_OVER_EPS0 = 1.602176634e-19 / 8.8541878128e-12 * 1e9
# Boltzmann constant, eV/K
KB = 8.617333262e-5


def link_permittivity(e1, e2):
    """Harmonic mean of the permittivities of the two nodes of a link."""
    return 2.0 * e1 * e2 / (e1 + e2)


def poisson_operator(shape, h, eps_r):
    """The symmetric matrix L of sum over links (i, j) of c_ij (phi_i - phi_j)^2 / 2,
    c_ij = link permittivity / h^2: (L phi)_i = sum_j c_ij (phi_i - phi_j) over the
    neighbours j of i inside the box (no term for links leaving it)."""
    px, py, pz = shape
    n = px * py * pz
    idx = np.arange(n).reshape(shape)
    eps = np.asarray(eps_r, dtype=float).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for axis in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[axis] = slice(0, shape[axis] - 1)
        b[axis] = slice(1, shape[axis])
        i = idx[tuple(a)].ravel()
        j = idx[tuple(b)].ravel()
        c = link_permittivity(eps[tuple(a)].ravel(), eps[tuple(b)].ravel()) / h ** 2
        rows += [i, j]
        cols += [j, i]
        vals += [-c, -c]
        np.add.at(diag, i, c)
        np.add.at(diag, j, c)
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def poisson_solve(shape, h, eps_r, dirichlet, phi_fixed, rho):
    """phi on the P grid: (L phi)_i = (e/eps0) rho_i at free nodes, phi = phi_fixed at
    Dirichlet nodes.  Needs at least one Dirichlet node (else phi is fixed only up to
    a constant)."""
    L = poisson_operator(shape, h, eps_r)
    d = np.asarray(dirichlet, dtype=bool).ravel()
    if not d.any():
        raise ValueError("at least one Dirichlet node is needed")
    f = ~d
    phi = np.where(d, np.asarray(phi_fixed, dtype=float).ravel(), 0.0)
    b = E_OVER_EPS0 * np.asarray(rho, dtype=float).ravel()[f] - L[f][:, d] @ phi[d]
    phi[f] = spla.spsolve(L[f][:, f].tocsc(), b)
    return phi.reshape(shape)


def occupancy(E, n_holes, T, iters=200):
    """Fermi-Dirac occupations f_n and the level mu with sum f_n = n_holes, mu found by
    bisection (the sum decreases monotonically as mu falls)."""
    E = np.asarray(E, dtype=float)
    if not 0.0 <= n_holes <= len(E):
        raise ValueError("0 <= n_holes <= number of states")
    kT = KB * T

    def f_of(mu):
        return 0.5 * (1.0 - np.tanh((E - mu) / (2.0 * kT)))   # = 1/(1+exp((E-mu)/kT))

    lo, hi = E.min() - 60.0 * kT - 1.0, E.max() + 60.0 * kT + 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if f_of(mid).sum() > n_holes:
            hi = mid
        else:
            lo = mid
    mu = 0.5 * (lo + hi)
    return f_of(mu), mu


def hole_density(psi_j, f, shape, h):
    """p(r) = sum_n f_n sum_c |psi_n,c(r)|^2 / h^3 on the Schroedinger grid; psi_j is
    (6N, nev) with index 6 p + c (either basis: the sum over c is invariant)."""
    nev = psi_j.shape[1]
    dens = (np.abs(np.asarray(psi_j)) ** 2).reshape(-1, 6, nev).sum(axis=1)   # (N, nev)
    return (dens @ np.asarray(f, dtype=float)).reshape(shape) / h ** 3


def embed(small, big_shape, offset):
    """A P-grid array holding `small` at the offset and zero elsewhere."""
    out = np.zeros(big_shape)
    ox, oy, oz = offset
    nx, ny, nz = small.shape
    out[ox:ox + nx, oy:oy + ny, oz:oz + nz] = small
    return out


def restrict(big, small_shape, offset):
    ox, oy, oz = offset
    nx, ny, nz = small_shape
    return big[ox:ox + nx, oy:oy + ny, oz:oz + nz]


class Anderson:
    """Anderson mixing with a history of the last m (input, residual) pairs."""

    def __init__(self, mixing, m):
        self.mixing, self.m = mixing, m
        self.hist_x, self.hist_F = [], []

    def step(self, x, F):
        nxt = anderson_step(x, F, self.hist_x, self.hist_F, self.mixing, self.m)
        self.hist_x.append(x)
        self.hist_F.append(F)
        excess = max(0, len(self.hist_x) - self.m)
        del self.hist_x[:excess], self.hist_F[:excess]
        return nxt


def anderson_step(x, F, hist_x, hist_F, mixing, m):
    """Next input from the current input x and residual F, given the previous
    inputs and residuals (lists, oldest first; at most m are used)."""
    if m == 0 or not hist_x:
        return x + mixing * F
    xs = hist_x[-m:] + [x]
    Fs = hist_F[-m:] + [F]
    dX = np.stack([(xs[k + 1] - xs[k]).ravel() for k in range(len(xs) - 1)], axis=1)
    dF = np.stack([(Fs[k + 1] - Fs[k]).ravel() for k in range(len(Fs) - 1)], axis=1)
    g, *_ = np.linalg.lstsq(dF, F.ravel(), rcond=None)
    return x + mixing * F - ((dX + mixing * dF) @ g).reshape(x.shape)


def sp_loop(grid, nev, V_off, pshape, offset, eps_r, dirichlet, phi_fixed, n_holes, T,
            strain=None, B=(0.0, 0.0, 0.0), rho_fixed=None, mixing=0.3, history=5, tol=1e-8,
            max_iter=100, phi0=None, material=SI_MATERIAL, method="auto"):
    """Self-consistent Schroedinger-Poisson loop (Fig. 2a).

    Starts from phi0 or, if None, from the hole-free potential (Poisson with
    rho_fixed only).  Each iteration: V = V_off + phi_in on the Schroedinger grid;
    lowest nev eigenpairs of H(V); occupations; hole density; Poisson for phi_out;
    stop if max |phi_out - phi_in| <= tol, else mix (Anderson over `history`
    previous iterations, damping `mixing`).  Returns a dict with phi (the
    last phi_in), E, psi_j, f, mu, density (Schroedinger grid), iterations, delta
    (the last max |phi_out - phi_in|) and converged."""
    if not isinstance(grid, Grid):
        grid = Grid(*grid)
    sshape = grid.shape
    rho0 = np.zeros(pshape) if rho_fixed is None else np.asarray(rho_fixed, dtype=float)
    if phi0 is None:
        phi_in = poisson_solve(pshape, grid.h, eps_r, dirichlet, phi_fixed, rho0)
    else:
        phi_in = np.array(phi0, dtype=float)
    delta = np.inf
    mixer = Anderson(mixing, history)
    for it in range(1, max_iter + 1):
        V = np.asarray(V_off, dtype=float) + restrict(phi_in, sshape, offset)
        E, psi, _ = solve_lowest(grid, material, nev, V=V, strain=strain, B=B, method=method)
        f, mu = occupancy(E, n_holes, T)
        p = hole_density(psi, f, sshape, grid.h)
        phi_out = poisson_solve(pshape, grid.h, eps_r, dirichlet, phi_fixed,
                                rho0 + embed(p, pshape, offset))
        delta = float(np.abs(phi_out - phi_in).max())
        out = dict(phi=phi_in, E=E, psi_j=psi, f=f, mu=mu, density=p, iterations=it,
                   delta=delta, converged=delta <= tol)
        if out["converged"]:
            break
        phi_in = mixer.step(phi_in, phi_out - phi_in)
    return out
