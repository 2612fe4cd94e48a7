"""Pins of the oracle's g-matrices and the effective two-spin model (CPU only).

What fixes them independently of the oracle's own formulas:
  * closed forms at a single grid point: the heavy-hole doublet under biaxial
    strain (g = diag(0, 0, 6 kappa)) and the split-off doublet (g_sym = (4 kappa - 2) 1);
  * the Zeeman splitting of the full Hamiltonian at small B, diagonalised
    densely, against mu_B |g B| (degenerate perturbation theory);
  * invariants: the gauge origin and the doublet basis do not change what is
    physical, time reversal makes tr M_b vanish, a mirror-symmetric double dot
    has mirror-image g-tensors;
  * the paper's worked example t = Delta / sqrt(2);
  * closed forms of Eq. HB and of J_perp, J_par.
"""

import pathlib

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid, hamiltonian_j
from oracle.constants import MU_B
from oracle.gmatrix import (anisotropic_exchange, centre_of_charge, double_dot_g, doublet_g,
                            effective_hamiltonian, field_derivative, g_matrix, qubit_frame,
                            rotation, symmetric_g, tunnel_coupling, two_spin_model,
                            u_minus_eps, zeeman_fields, zeeman_trace)
from oracle.solve import lowest_dense

KAPPA = SI_MATERIAL["kappa"]
GOLDEN = pathlib.Path(__file__).parent / "golden"


def _dot(grid, seed, strain=True, centre=(0.0, 0.0, 0.0)):
    """A smooth confining potential with a little disorder, and random strain."""
    rng = np.random.default_rng(seed)
    x, y, z = grid.coords()
    c = grid.centre() + np.asarray(centre)
    V = 0.02 * ((x - c[0]) ** 2 + 1.3 * (y - c[1]) ** 2 + 0.8 * (z - c[2]) ** 2)
    V = V.ravel() + rng.normal(0.0, 2e-3, grid.npts)
    S = rng.normal(0.0, 2e-3, (grid.npts, 6)) if strain else None
    return V, S


def _lowest(grid, nev, V, S, B=(0.0, 0.0, 0.0)):
    H = hamiltonian_j(grid, SI_MATERIAL, V=V, strain=S, B=B)
    return lowest_dense(H, nev)


def test_heavy_hole_doublet_closed_form():
    """One grid point, biaxial strain: |3/2, +-3/2> are exact eigenstates, and
    2 kappa mu_B B.J within them gives g = diag(0, 0, 6 kappa)."""
    g1 = Grid(1, 1, 1, 0.5)
    S = np.array([[-0.01, -0.01, 0.006, 0.0, 0.0, 0.0]])
    H = hamiltonian_j(g1, SI_MATERIAL, V=np.zeros(1), strain=S).toarray()
    u = np.zeros((6, 2), dtype=complex)
    u[0, 0] = u[3, 1] = 1.0
    assert np.abs(H @ u - u * np.diag(u.conj().T @ H @ u).real).max() < 1e-15
    D = field_derivative(g1, SI_MATERIAL, np.zeros(1), S)
    g = g_matrix(u, D)
    expect = np.zeros((3, 3))
    expect[2, 2] = 6.0 * KAPPA
    assert np.abs(g - expect).max() < 1e-9
    assert np.abs(symmetric_g(g) - np.diag([0.0, 0.0, 6.0 * abs(KAPPA)])).max() < 1e-9


def test_split_off_doublet_is_isotropic():
    """One grid point, no strain: the Gamma7 doublet |1/2, +-1/2> at +Delta has the
    Lande factor of j = 1/2 from l = 1, s = 1/2: g_sym = (4 kappa - 2) 1."""
    g1 = Grid(1, 1, 1, 0.5)
    H = hamiltonian_j(g1, SI_MATERIAL, V=np.zeros(1)).toarray()
    u = np.zeros((6, 2), dtype=complex)
    u[4, 0] = u[5, 1] = 1.0
    E = np.diag(u.conj().T @ H @ u).real
    assert np.abs(H @ u - u * E).max() < 1e-15
    assert abs(E[0] - H[0, 0].real - SI_MATERIAL["delta_so"]) < 1e-15   # Gamma7 at +Delta
    g = g_matrix(u, field_derivative(g1, SI_MATERIAL, np.zeros(1)))
    assert np.abs(np.linalg.svd(g, compute_uv=False) - abs(4 * KAPPA - 2)).max() < 1e-9
    assert np.abs(symmetric_g(g) - (4 * KAPPA - 2) * np.eye(3)).max() < 1e-9


def test_g_matrix_gives_the_zeeman_splitting_of_the_full_hamiltonian():
    """Orbital (Peierls) and spin parts together: the lowest doublet of H(B),
    diagonalised densely at small B, splits by mu_B |g B| (Richardson in |B|)."""
    grid = Grid(5, 4, 4, 0.5)
    V, S = _dot(grid, 3)
    E, psi = _lowest(grid, 2, V, S)
    g, _, tr = doublet_g(grid, SI_MATERIAL, psi, V, S)
    assert np.abs(tr).max() < 1e-10 * np.abs(g).max()
    rng = np.random.default_rng(7)
    beta = 2e-3
    for _ in range(3):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        s1 = np.diff(_lowest(grid, 2, V, S, B=tuple(beta * n))[0])[0] / beta
        s2 = np.diff(_lowest(grid, 2, V, S, B=tuple(2 * beta * n))[0])[0] / (2 * beta)
        slope = (4.0 * s1 - s2) / 3.0
        expect = MU_B * np.linalg.norm(g @ n)
        assert abs(slope - expect) < 1e-6 * expect, (slope, expect)


def test_eigen_doublet_g_is_independent_of_gauge_origin_and_basis():
    grid = Grid(5, 4, 3, 0.5)
    V, S = _dot(grid, 11)
    _, psi = _lowest(grid, 2, V, S)
    D0 = field_derivative(grid, SI_MATERIAL, V, S)
    D1 = field_derivative(grid, SI_MATERIAL, V, S, origin=(1.3, -0.7, 0.4))
    g0, g1 = g_matrix(psi, D0), g_matrix(psi, D1)
    assert np.abs(g0 - g1).max() < 1e-9 * np.abs(g0).max()
    assert np.abs(zeeman_trace(psi, D0)).max() < 1e-10 * np.abs(g0).max()
    # a unitary change of the doublet basis rotates g on the left by a proper rotation
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)))
    g2 = g_matrix(psi @ Q, D0)
    R = g2 @ np.linalg.inv(g0)
    assert np.abs(R @ R.T - np.eye(3)).max() < 1e-8 and abs(np.linalg.det(R) - 1) < 1e-8
    assert np.abs(symmetric_g(g2) - symmetric_g(g0)).max() < 1e-8 * np.abs(g0).max()


def test_mirror_symmetric_double_dot():
    """V(-x) = V(x), no strain: the localised doublets sit at mirror-image centres and
    their g-tensors are mirror images, g_R = P g_L P with P = diag(1, -1, -1) (field and
    spin are axial vectors); the eigen-doublets obey time reversal."""
    grid = Grid(14, 4, 4, 0.5)
    x, _, _ = grid.coords()
    X = x - grid.centre()[0]
    V = (0.2 * (np.abs(X) < 0.8) + 0.02 * (np.abs(X) - 2.2) ** 2).ravel()   # two wells, a barrier
    E, psi = _lowest(grid, 6, V, None)
    assert E[2] - E[0] < 0.2 * (E[4] - E[0])   # bonding and antibonding well below the rest
    psi, E = psi[:, :4], E[:4]
    out = double_dot_g(grid, SI_MATERIAL, psi, E, V, None)
    cL, cR = out["centre"][2], out["centre"][3]
    assert cL[0] < 0 < cR[0]
    assert abs(cL[0] + cR[0]) < 1e-9 and np.abs(cL[1:] - cR[1:]).max() < 1e-9
    P = np.diag([1.0, -1.0, -1.0])
    gL, gR = out["g_sym"][2], out["g_sym"][3]
    assert np.abs(gR - P @ gL @ P).max() < 1e-8 * np.abs(gL).max()
    for k in (0, 1):
        assert np.abs(out["trace"][k]).max() < 1e-9 * np.abs(out["g"][k]).max()
    assert out["delta"] > 0 and abs(out["t"] - out["delta"] / np.sqrt(2)) < 1e-18
    assert abs(out["d"] - (cR[0] - cL[0])) < 1e-9


def test_tunnel_coupling_worked_example():
    """The paper's bonding/antibonding energies at zero detuning give t = 1.13e-5 eV."""
    vals = {}
    for line in (GOLDEN / "tunnel_coupling_symmetric_dqd.txt").read_text().splitlines():
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    t = tunnel_coupling(vals["E_bonding_eV"] - vals["E_antibonding_eV"])
    assert float(f"{t:.3g}") == vals["t_eV"]


def test_effective_hamiltonian_closed_forms():
    rng = np.random.default_rng(5)
    t, J = 1.13e-5, 2.0e-7
    Ue = u_minus_eps(t, J)
    assert abs(2 * t * t / Ue - J) < 1e-22
    # B = 0: three triplets at 0, the singlets mixed by sqrt(2) t
    H = effective_hamiltonian(Ue, t, np.zeros(3), np.zeros(3))
    ev = np.linalg.eigvalsh(H)
    r = np.sqrt(Ue * Ue / 4 + 2 * t * t)
    expect = np.sort([Ue / 2 - r, 0, 0, 0, Ue / 2 + r])
    assert np.abs(ev - expect).max() < 1e-18
    # the S(1,1)-T gap is J to first order in J / (U - eps)
    assert abs((0 - ev[0]) - J) < 2 * J * J / Ue
    # identical isotropic g, no spin-orbit rotation: the triplets split by mu_B g |B|
    g0 = 1.7
    B = rng.normal(size=3)
    bbar, db = zeeman_fields(g0 * np.eye(3), g0 * np.eye(3), 0.0, (0, 0, 1), B)
    assert np.abs(db).max() == 0.0
    H = effective_hamiltonian(Ue, t, bbar, db)
    assert np.abs(H - H.conj().T).max() == 0.0
    ev = np.linalg.eigvalsh(H)
    bz = MU_B * g0 * np.linalg.norm(B)
    expect = np.sort([Ue / 2 - r, -bz, 0, bz, Ue / 2 + r])
    assert np.abs(ev - expect).max() < 1e-18
    # a spin-orbit axis along B rotates nothing: delta_b vanishes
    _, db = zeeman_fields(g0 * np.eye(3), g0 * np.eye(3), 0.3, B, B)
    assert np.abs(db).max() < 1e-14 * MU_B * g0 * np.linalg.norm(B)


def test_anisotropic_exchange_closed_forms():
    J, th = 3e-7, 0.37
    g = 1.4 * np.eye(3)
    B = np.array([0.0, 0.0, 0.05])
    # spin-orbit axis along the field: the flip-flop and Ising parts are both J
    _, _, perp, par = anisotropic_exchange(J, th, (0, 0, 1), g, g, B)
    assert abs(perp - J) < 1e-20 and abs(par - J) < 1e-20
    # perpendicular: J_par = J cos(2 theta), |J_perp| = J cos^2(theta)
    _, _, perp, par = anisotropic_exchange(J, th, (1, 0, 0), g, g, B)
    assert abs(par - J * np.cos(2 * th)) < 1e-20
    assert abs(perp - J * np.cos(th) ** 2) < 1e-20
    # the frames' freedom about z changes neither
    rng = np.random.default_rng(9)
    gL = symmetric_g(rng.normal(size=(3, 3)))
    gR = symmetric_g(rng.normal(size=(3, 3)))
    Bv = rng.normal(size=3)
    n = rng.normal(size=3)
    _, _, p0, q0 = anisotropic_exchange(J, th, n, gL, gR, Bv)
    RL = rotation((0, 0, 1), 0.9) @ qubit_frame(gL @ Bv)
    RR = rotation((0, 0, 1), -2.1) @ qubit_frame(gR @ Bv)
    _, _, p1, q1 = anisotropic_exchange(J, th, n, gL, gR, Bv, RL, RR)
    assert abs(p0 - p1) < 1e-18 and abs(q0 - q1) < 1e-18
    # J_par is n_L . J_hat n_R whatever the frames
    nL = gL @ Bv / np.linalg.norm(gL @ Bv)
    nR = gR @ Bv / np.linalg.norm(gR @ Bv)
    assert abs(q0 - nL @ (J * rotation(n, -2 * th)) @ nR) < 1e-20


@pytest.mark.parametrize("n", [(0, 0, 1), (0, 0, -1), (1, 2, -3), (1e-9, 0, -1)])
def test_qubit_frame_is_a_rotation_onto_z(n):
    R = qubit_frame(n)
    n = np.asarray(n, dtype=float) / np.linalg.norm(n)
    assert np.abs(R @ n - np.array([0, 0, 1])).max() < 1e-12
    assert np.abs(R @ R.T - np.eye(3)).max() < 1e-12 and abs(np.linalg.det(R) - 1) < 1e-12


def test_two_spin_model_collects_the_pieces():
    rng = np.random.default_rng(4)
    gL = symmetric_g(rng.normal(size=(3, 3)))
    gR = symmetric_g(rng.normal(size=(3, 3)))
    out = two_spin_model(gL, gR, 1.1e-5, 2.3e-7, 0.2, (0, 1, 0), (0.02, -0.01, 0.03))
    assert abs(out["dEz"] - np.linalg.norm(out["db"])) < 1e-20
    assert np.abs(np.linalg.eigvalsh(out["H"]) - out["E"]).max() == 0.0
    assert out["J_perp"] >= 0


def test_centre_of_charge_follows_a_displaced_dot():
    """A dot pushed to +x and its mirror image at -x: opposite centres along x."""
    grid = Grid(9, 3, 3, 0.5)
    r = []
    for sx in (1.0, -1.0):
        x, y, z = grid.coords()
        c = grid.centre()
        V = (0.05 * (x - c[0] - sx) ** 2 + 0.02 * (y - c[1]) ** 2).ravel()
        _, psi = _lowest(grid, 2, V, None)
        r.append(centre_of_charge(grid, psi))
    assert r[0][0] > 0.1
    assert abs(r[0][0] + r[1][0]) < 1e-10 and np.abs(r[0][1:] - r[1][1:]).max() < 1e-10


def test_field_derivative_is_the_zeeman_term_plus_a_position_commutator_form():
    """For straight-link Peierls phases in the symmetric gauge (the two-step links of
    the mixed derivatives average to the straight one at first order in B),
    dH/dB_b = Z_b + i (e / 2 hbar) eps_bcd R_c H_0 R_d, R the position about the gauge
    origin and Z_b the on-site Zeeman matrix per tesla."""
    from oracle.constants import E_OVER_HBAR
    from oracle.hamiltonian import U_J_FROM_LS, onsite_so_zeeman_ls
    import scipy.sparse as sp
    grid = Grid(4, 3, 3, 0.5)
    V, S = _dot(grid, 21)
    origin = np.array([0.4, -0.3, 0.2])
    D = field_derivative(grid, SI_MATERIAL, V, S, origin=origin)
    H0 = hamiltonian_j(grid, SI_MATERIAL, V=V, strain=S).toarray()
    x, y, z = grid.coords()
    c = grid.centre() + origin
    R = [np.repeat((q - c[k]).ravel(), 6) for k, q in enumerate((x, y, z))]
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    for b in range(3):
        e = np.zeros(3)
        e[b] = 1.0
        hz = onsite_so_zeeman_ls(SI_MATERIAL, e) - onsite_so_zeeman_ls(SI_MATERIAL)
        Z = sp.kron(sp.identity(grid.npts), U_J_FROM_LS @ hz @ U_J_FROM_LS.conj().T).toarray()
        orb = sum(eps[b, cc, d] * (R[cc][:, None] * H0 * R[d][None, :])
                  for cc in range(3) for d in range(3))
        expect = Z + 0.5j * E_OVER_HBAR * orb
        # the difference quotients lose about 1e-15 eV / (12 s) to rounding
        assert np.abs(D[b].toarray() - expect).max() < 1e-9 * np.abs(expect).max()
