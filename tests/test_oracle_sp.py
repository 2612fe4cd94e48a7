"""Pins of the oracle's electrostatics and self-consistent loop (CPU only).

Each check compares the oracle with something other than itself: continuum
closed forms that second-order finite differences reproduce exactly, a
conservation law summed with independent code, symmetry, the Fermi-Dirac
closed form, and the physics of the loop (no holes: one pass; holes repel).
"""

import numpy as np
import pytest

from oracle import (E_OVER_EPS0, Grid, hole_density, occupancy, poisson_solve, sp_loop,
                    solve_lowest, SI_MATERIAL, to_j_basis)
from oracle.poisson import KB
from synth import sp_device


def test_constants():
    # e / eps0 = 1.602176634e-19 C / 8.8541878128e-12 F/m = 1.80951e-8 V m
    assert abs(E_OVER_EPS0 - 18.0951282) < 1e-6
    assert abs(KB * 11604.518 - 1.0) < 1e-6          # 1 eV = 11604.518 K


@pytest.mark.parametrize("cross", [(1, 1), (3, 4)])
def test_poisson_uniform_charge_between_two_plates(cross):
    """-eps phi'' = (e/eps0) rho between plates at phi = a (x = 0) and b (x = L):
    phi = a + (b - a) x / L + (e/eps0) rho x (L - x) / (2 eps).  Second differences
    are exact on quadratics, so the nodes carry the continuum values; the
    field-free side faces make every (y, z) column the same."""
    n, h, eps, rho0, a, b = 21, 0.5, 3.9, 2e-3, -0.2, 0.1
    shape = (n,) + cross
    dirichlet = np.zeros(shape, dtype=bool)
    dirichlet[0] = dirichlet[-1] = True
    phi_fixed = np.zeros(shape)
    phi_fixed[0], phi_fixed[-1] = a, b
    rho = np.full(shape, rho0)
    phi = poisson_solve(shape, h, np.full(shape, eps), dirichlet, phi_fixed, rho)
    x = np.arange(n) * h
    L = (n - 1) * h
    exact = a + (b - a) * x / L + E_OVER_EPS0 * rho0 * x * (L - x) / (2 * eps)
    assert np.abs(phi - exact[:, None, None]).max() < 1e-12


def test_poisson_two_dielectrics_in_series():
    """No charge, plates at 0 and V, eps1 on nodes 0..m-1 and eps2 on nodes m..n-1:
    the interface lies midway between nodes m-1 and m, D is uniform, and the
    continuum potential (slope D/eps on each side) is what the nodes must hold."""
    n, m, h, e1, e2, V = 17, 6, 0.4, 11.7, 3.9, 0.25
    shape = (n, 2, 3)
    eps = np.full(shape, e2)
    eps[:m] = e1
    dirichlet = np.zeros(shape, dtype=bool)
    dirichlet[0] = dirichlet[-1] = True
    phi_fixed = np.zeros(shape)
    phi_fixed[-1] = V
    phi = poisson_solve(shape, h, eps, dirichlet, phi_fixed, np.zeros(shape))
    x = np.arange(n) * h
    xi, L = (m - 0.5) * h, (n - 1) * h
    D = V / (xi / e1 + (L - xi) / e2)
    exact = np.where(x <= xi, D * x / e1, D * xi / e1 + D * (x - xi) / e2)
    assert np.abs(phi - exact[:, None, None]).max() < 1e-12


def test_poisson_gauss_law_and_node_equations():
    """Random permittivity, charge and electrodes: every free node's equation holds
    (summed over its in-box neighbours by an explicit loop), and the charge of the
    free nodes equals the flux into the electrodes (free-free links cancel in the
    sum of all equations; no flux leaves through the other faces)."""
    rng = np.random.default_rng(3)
    shape, h = (7, 6, 5), 0.5
    eps = rng.uniform(1.0, 12.0, shape)
    rho = rng.normal(0.0, 1e-2, shape)
    dirichlet = np.zeros(shape, dtype=bool)
    dirichlet[2:5, :, -1] = True
    dirichlet[0, 0, 0] = True
    phi_fixed = np.where(dirichlet, rng.uniform(-0.3, 0.3, shape), 0.0)
    phi = poisson_solve(shape, h, eps, dirichlet, phi_fixed, rho)
    assert np.all(phi[dirichlet] == phi_fixed[dirichlet])
    flux = 0.0
    for i in range(shape[0]):
        for j in range(shape[1]):
            for k in range(shape[2]):
                if dirichlet[i, j, k]:
                    continue
                s = 0.0
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1),
                                   (0, 0, -1)):
                    a, b, c = i + di, j + dj, k + dk
                    if not (0 <= a < shape[0] and 0 <= b < shape[1] and 0 <= c < shape[2]):
                        continue
                    e = 2 * eps[i, j, k] * eps[a, b, c] / (eps[i, j, k] + eps[a, b, c])
                    t = e * (phi[i, j, k] - phi[a, b, c]) / h ** 2
                    s += t
                    if dirichlet[a, b, c]:
                        flux += t
                assert abs(s - E_OVER_EPS0 * rho[i, j, k]) < 1e-10
    assert abs(flux - E_OVER_EPS0 * rho[~dirichlet].sum()) < 1e-9


def test_poisson_mirror_symmetry():
    d = sp_device("sp_dqd_small")
    rho = np.zeros(d.pshape)
    rho[10:20, 5:9, 4:9] = 1e-3
    rho = 0.5 * (rho + rho[::-1])
    phi = poisson_solve(d.pshape, d.h, d.eps_r, d.dirichlet, d.phi_fixed, rho)
    assert np.abs(phi - phi[::-1]).max() < 1e-12


def test_poisson_needs_an_electrode():
    shape = (4, 4, 4)
    with pytest.raises(ValueError):
        poisson_solve(shape, 0.5, np.ones(shape), np.zeros(shape, bool), np.zeros(shape),
                      np.zeros(shape))


def test_occupancy_closed_forms():
    T = 1.5
    kT = KB * T
    # two states, one hole: mu is the midpoint and f0 = 1 / (1 + exp(-dE / 2kT))
    E = np.array([0.010, 0.0101])
    f, mu = occupancy(E, 1.0, T)
    assert abs(mu - 0.01005) < 1e-14
    assert abs(f[0] - 1.0 / (1.0 + np.exp(-0.0001 / (2 * kT)))) < 1e-12
    # Kramers pairs 5 meV apart, two holes: mu sits midway between the two lowest
    # pairs (f(-x) + f(x) = 1; the third pair, 38 kT higher still, adds < 1e-16)
    E = np.repeat([0.1, 0.105, 0.11], 2)
    f, mu = occupancy(E, 2.0, T)
    assert abs(mu - 0.1025) < 1e-9     # the count fixes mu only to ~1e-12 here
    f1 = 1.0 / (1.0 + np.exp(0.0025 / kT))
    assert np.allclose(f, [1 - f1, 1 - f1, f1, f1, 0, 0], rtol=1e-9, atol=1e-15)
    # the count is met for any filling and temperature
    rng = np.random.default_rng(0)
    E = np.sort(rng.uniform(0, 0.01, 9))
    for n_h in (0.5, 2.0, 4.3):
        for T in (1.5, 30.0):
            f, _ = occupancy(E, n_h, T)
            assert abs(f.sum() - n_h) < 1e-12


def test_anderson_on_a_linear_map():
    """On a linear fixed-point problem x = M x + c in n dimensions, Anderson mixing
    with a history of at least n terminates after n + 1 steps (it is then GMRES;
    Walker and Ni, SIAM J. Numer. Anal. 49, 1715 (2011)); with no history it is
    plain damped iteration x + a F."""
    from oracle.poisson import Anderson
    rng = np.random.default_rng(7)
    n = 4
    M = rng.normal(0.0, 0.6, (n, n))
    c = rng.normal(size=n)
    exact = np.linalg.solve(np.eye(n) - M, c)
    mixer = Anderson(0.5, 5)
    x = np.zeros(n)
    for _ in range(n + 1):
        x = mixer.step(x, M @ x + c - x)
    assert np.abs(x - exact).max() < 1e-9
    assert len(mixer.hist_x) == 5
    lin = Anderson(0.5, 0)
    y = rng.normal(size=n)
    F = M @ y + c - y
    assert np.array_equal(lin.step(y, F), y + 0.5 * F)


def test_hole_density_counts_the_holes_in_either_basis():
    """sum p h^3 = n_holes for normalised states; sum_c |psi_c|^2 is the same in the
    |L S> and |J m_j> bases (U is unitary)."""
    d = sp_device("sp_tiny")
    g = Grid(*d.shape, d.h)
    E, psi_j, H = solve_lowest(g, SI_MATERIAL, 8, V=d.V_off)
    f, _ = occupancy(E, 2.0, 1.5)
    p = hole_density(psi_j, f, d.shape, d.h)
    assert abs(p.sum() * d.h ** 3 - 2.0) < 1e-10
    # |L S> eigenvectors of the same H: the density does not change
    from oracle import lowest_dense
    _, psi_ls = lowest_dense(H, 8)
    assert np.abs(to_j_basis(psi_ls) - psi_ls).max() > 1e-3   # the bases differ ...
    p_ls = hole_density(psi_ls, f, d.shape, d.h)
    assert np.abs(p_ls - p).max() < 1e-9 * p.max()           # ... the density does not


def _loop(d, n_holes, **kw):
    kw.setdefault("tol", 1e-9)
    return sp_loop(Grid(*d.shape, d.h), d.nev, d.V_off, d.pshape, d.offset, d.eps_r,
                   d.dirichlet, d.phi_fixed, n_holes, d.T, strain=d.strain, B=d.B,
                   method="arpack", **kw)


def test_sp_loop_without_holes_is_one_poisson_solve():
    """No holes: the density vanishes, the first output equals the input (the
    hole-free potential) and the eigenvalues are those of V_off + phi_Laplace."""
    d = sp_device("sp_tiny")
    r = _loop(d, 0.0)
    assert r["converged"] and r["iterations"] == 1 and r["delta"] < 1e-12
    phi0 = poisson_solve(d.pshape, d.h, d.eps_r, d.dirichlet, d.phi_fixed, np.zeros(d.pshape))
    assert np.abs(r["phi"] - phi0).max() < 1e-14


def test_sp_loop_fixed_point_and_repulsion():
    """Two holes: the loop reaches a potential that reproduces itself (one more
    Schroedinger-density-Poisson pass changes it by <= tol), the holes raise
    the potential energy of their own states (Coulomb repulsion), and the
    density integrates to two holes."""
    d = sp_device("sp_tiny")
    tol = 1e-9
    r = _loop(d, 2.0, tol=tol)
    assert r["converged"], r["delta"]
    g = Grid(*d.shape, d.h)
    from oracle import embed, restrict
    E, psi, _ = solve_lowest(g, SI_MATERIAL, d.nev, V=d.V_off + restrict(r["phi"], d.shape,
                                                                         d.offset),
                             method="arpack")
    f, _ = occupancy(E, 2.0, d.T)
    phi_out = poisson_solve(d.pshape, d.h, d.eps_r, d.dirichlet, d.phi_fixed,
                            embed(hole_density(psi, f, d.shape, d.h), d.pshape, d.offset))
    assert np.abs(phi_out - r["phi"]).max() <= tol * 1.01
    assert np.abs(E - r["E"]).max() < 1e-10
    r0 = _loop(d, 0.0)
    assert r["E"][0] > r0["E"][0] + 1e-3
    assert np.all(r["phi"] >= r0["phi"] - 1e-12)      # positive charge raises phi everywhere
    assert abs(r["density"].sum() * d.h ** 3 - 2.0) < 1e-9


def test_sp_loop_mirror_symmetric_device():
    """A device symmetric under x -> -x (B = 0, no strain) converges to a
    mirror-symmetric potential and density."""
    d = sp_device("sp_tiny")
    assert np.array_equal(d.dirichlet, d.dirichlet[::-1])
    r = _loop(d, 2.0)
    assert r["converged"]
    assert np.abs(r["phi"] - r["phi"][::-1]).max() < 1e-8
    assert np.abs(r["density"] - r["density"][::-1]).max() < 1e-6 * r["density"].max()


def test_anderson_and_linear_mixing_reach_the_same_fixed_point():
    d = sp_device("sp_tiny")
    a = _loop(d, 2.0, history=5, mixing=0.3)
    b = _loop(d, 2.0, history=0, mixing=0.1, max_iter=400)
    assert a["converged"] and b["converged"]
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-7
    assert np.abs(a["E"] - b["E"]).max() < 1e-8
