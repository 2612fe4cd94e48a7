"""Pins of the CPU oracle against closed forms, invariants and brute force.

Each closed form below is written out here from the mathematics (not taken from
the oracle), so that a dropped term, a wrong sign, index or transposed operand
in the oracle's assembly fails at least one test.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import (E0, MU_B, SI_MATERIAL, Grid, U_J_FROM_LS, hamiltonian_j,
                    hamiltonian_ls, hf_gradient, lowest_arpack, lowest_dense,
                    onsite_so_zeeman_ls, strain_orbital_ls, gate_potential)

SI = dict(SI_MATERIAL)


def _lh_so_pair(P, Q, D):
    """Eigenvalues of [[P - Q, -sqrt2 Q], [-sqrt2 Q, P + D]] (the coupled
    light-hole / split-off pair when R = S = 0)."""
    m = P + (D - Q) / 2.0
    r = np.sqrt(((D + Q) / 2.0) ** 2 + 2.0 * Q ** 2)
    return m - r, m + r


def _axial_spectrum(P, Q, D):
    """Full 6-level spectrum of a Luttinger-type matrix with R = S = 0."""
    lo, hi = _lh_so_pair(P, Q, D)
    return np.sort([P + Q, P + Q, lo, lo, hi, hi])


def _bloch_block(H, grid, q):
    """6x6 matrix of H between plane waves e^{i q.r} (x) e_c on a periodic grid,
    and the norm of the part of H e_q v that leaves the plane-wave subspace."""
    x, y, z = grid.coords()
    ph = np.exp(1j * (q[0] * x + q[1] * y + q[2] * z)).ravel()
    N = grid.npts
    cols = []
    for c in range(6):
        v = np.zeros((N, 6), dtype=complex)
        v[:, c] = ph
        cols.append((H @ v.ravel()).reshape(N, 6))
    Hq = np.array([[np.vdot(ph, cols[c][:, cp]) / N for c in range(6)] for cp in range(6)])
    # Hq[cp, c] = <e_q cp| H |e_q c>
    leak = 0.0
    for c in range(6):
        rebuilt = np.outer(ph, Hq[:, c])
        leak = max(leak, np.abs(cols[c] - rebuilt).max())
    return Hq, leak


def _random_fields(grid, seed, vscale=0.02, escale=2e-3):
    r = np.random.default_rng(seed)
    V = vscale * r.standard_normal(grid.npts)
    e = escale * r.standard_normal((grid.npts, 6))
    return V, e


# ----------------------------------------------------------------------------
# structure
# ----------------------------------------------------------------------------

def test_hermitian_and_symmetric_inner_products():
    g = Grid(5, 4, 3, 0.5)
    V, e = _random_fields(g, 1)
    H = hamiltonian_ls(g, SI, V, e, B=(0.4, -0.3, 0.8))
    assert abs(H - H.getH()).max() == 0.0
    r = np.random.default_rng(2)
    n = H.shape[0]
    x = r.standard_normal(n) + 1j * r.standard_normal(n)
    y = r.standard_normal(n) + 1j * r.standard_normal(n)
    a, b = np.vdot(x, H @ y), np.vdot(H @ x, y)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_u_is_unitary():
    assert np.abs(U_J_FROM_LS @ U_J_FROM_LS.conj().T - np.eye(6)).max() < 1e-15


@pytest.mark.parametrize("B", [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.2, -0.7, 0.45)])
def test_two_independent_assemblies_agree(B):
    """|L S> (DKK) form rotated by U equals the |J m_j> Luttinger-Kohn form."""
    g = Grid(4, 5, 3, 0.4)
    V, e = _random_fields(g, 3)
    Hl = hamiltonian_ls(g, SI, V, e, B)
    Hj = hamiltonian_j(g, SI, V, e, B)
    Uf = sp.kron(sp.identity(g.npts), U_J_FROM_LS)
    diff = abs(Uf @ Hl @ Uf.getH() - Hj).max()
    assert diff <= 1e-13 * abs(Hj).max()


def test_gamma3_121_variant_agrees_too():
    m = dict(SI, gamma3=1.21)
    g = Grid(3, 3, 4, 0.5)
    V, e = _random_fields(g, 4)
    Hl = hamiltonian_ls(g, m, V, e, (0.1, 0.2, 0.3))
    Hj = hamiltonian_j(g, m, V, e, (0.1, 0.2, 0.3))
    Uf = sp.kron(sp.identity(g.npts), U_J_FROM_LS)
    assert abs(Uf @ Hl @ Uf.getH() - Hj).max() <= 1e-13 * abs(Hj).max()


# ----------------------------------------------------------------------------
# bulk dispersion (periodic grid): discrete symbol vs closed forms
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("form", ["ls", "j"])
@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_bulk_dispersion_001(form, m):
    n, h = 8, 0.5
    g = Grid(n, n, n, h, periodic=True)
    H = (hamiltonian_ls if form == "ls" else hamiltonian_j)(g, SI)
    q = np.array([0.0, 0.0, 2 * np.pi * m / (n * h)])
    Hq, leak = _bloch_block(H, g, q)
    assert leak < 1e-12
    kz2 = (2 - 2 * np.cos(q[2] * h)) / h**2
    P = E0 * SI["gamma1"] * kz2
    Q = -2.0 * E0 * SI["gamma2"] * kz2
    ref = _axial_spectrum(P, Q, SI["delta_so"])
    got = np.linalg.eigvalsh(Hq)
    assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("form", ["ls", "j"])
@pytest.mark.parametrize("m", [1, 2, 3])
def test_bulk_dispersion_111(form, m):
    """Along [111] the problem is the [001] one with gamma2 -> gamma3
    (rotation about the body diagonal); discrete: P = 3 g1 k2, Q = -6 g3 s2."""
    n, h = 8, 0.5
    g = Grid(n, n, n, h, periodic=True)
    H = (hamiltonian_ls if form == "ls" else hamiltonian_j)(g, SI)
    qa = 2 * np.pi * m / (n * h)
    q = np.array([qa, qa, qa])
    Hq, leak = _bloch_block(H, g, q)
    assert leak < 1e-12
    k2 = (2 - 2 * np.cos(qa * h)) / h**2
    s2 = np.sin(qa * h) ** 2 / h**2
    P = E0 * 3.0 * SI["gamma1"] * k2
    Q = -6.0 * E0 * SI["gamma3"] * s2
    ref = _axial_spectrum(P, Q, SI["delta_so"])
    assert np.abs(np.linalg.eigvalsh(Hq) - ref).max() < 1e-12


def test_luttinger_masses_001_large_delta():
    """With the split-off band pushed far away (Delta = 100 eV) the [001]
    levels are the Luttinger heavy/light holes, g1 -+ 2 g2 in units of E0 k^2
    (k^2 the discrete (2 - 2 cos qh)/h^2), up to 2 Q^2 / Delta."""
    m = dict(SI, delta_so=100.0)
    n, h = 64, 0.5
    g = Grid(1, 1, n, h, periodic=True)
    qa = 2 * np.pi / (n * h)
    Hq, leak = _bloch_block(hamiltonian_ls(g, m), g, np.array([0, 0, qa]))
    assert leak < 1e-12
    w = np.linalg.eigvalsh(Hq)
    k2 = (2 - 2 * np.cos(qa * h)) / h**2
    assert abs(w[0] / (E0 * k2) - (m["gamma1"] - 2 * m["gamma2"])) < 1e-9
    Q = -2 * m["gamma2"] * E0 * k2
    lh = (m["gamma1"] + 2 * m["gamma2"]) * E0 * k2 - 2 * Q**2 / m["delta_so"]
    assert abs(w[2] - lh) / (E0 * k2) < 1e-9


def test_uniform_strain_periodic_q0():
    """q = 0 with uniform biaxial + uniaxial strain: P_e, Q_e closed form."""
    g = Grid(3, 3, 3, 0.5, periodic=True)
    exx = eyy = 0.0012
    ezz = -0.003
    e = np.tile([exx, eyy, ezz, 0, 0, 0], (g.npts, 1))
    for builder in (hamiltonian_ls, hamiltonian_j):
        H = builder(g, SI, None, e)
        Hq, leak = _bloch_block(H, g, np.zeros(3))
        assert leak < 1e-13
        P = -SI["a_v"] * (exx + eyy + ezz)
        Q = -(SI["b"] / 2.0) * (exx + eyy - 2 * ezz)
        ref = _axial_spectrum(P, Q, SI["delta_so"])
        assert np.abs(np.linalg.eigvalsh(Hq) - ref).max() < 1e-14


def test_shear_strain_111_closed_form():
    """Pure [111] shear e_xy = e_yz = e_xz = s: axial problem with Q = sqrt3 d s."""
    s = 7e-4
    D = strain_orbital_ls(SI, np.array([0, 0, 0, s, s, s]))
    Hs = np.kron(np.eye(2), D) + onsite_so_zeeman_ls(SI)
    ref = _axial_spectrum(0.0, np.sqrt(3) * SI["d"] * s, SI["delta_so"])
    assert np.abs(np.linalg.eigvalsh(Hs) - ref).max() < 1e-15


def test_compressive_strain_puts_light_hole_lowest():
    """e_zz = -0.3 %: the light-hole level lies below the heavy hole in hole
    energy (consistent with the LH-dominated states of the paper, Sec. III)."""
    D = strain_orbital_ls(SI, np.array([0, 0, -0.003, 0, 0, 0]))
    Hs = np.kron(np.eye(2), D) + onsite_so_zeeman_ls(SI)
    w, v = np.linalg.eigh(U_J_FROM_LS @ Hs @ U_J_FROM_LS.conj().T)
    ground = v[:, 0]
    lh_weight = abs(ground[1]) ** 2 + abs(ground[2]) ** 2
    assert lh_weight > 0.9


# ----------------------------------------------------------------------------
# hard walls and confinement
# ----------------------------------------------------------------------------

def test_hard_wall_chain():
    """nx = ny = 1: kx^2 = ky^2 = 2/h^2, all mixed terms vanish, kz^2 takes the
    Dirichlet values (2 - 2 cos(pi n/(nz+1)))/h^2."""
    nz, h = 12, 0.5
    g = Grid(1, 1, nz, h)
    H = hamiltonian_ls(g, SI).toarray()
    ref = []
    for n in range(1, nz + 1):
        lam = (2 - 2 * np.cos(np.pi * n / (nz + 1))) / h**2
        P = E0 * SI["gamma1"] * (4.0 / h**2 + lam)
        Q = E0 * SI["gamma2"] * (4.0 / h**2 - 2 * lam)
        ref.extend(_axial_spectrum(P, Q, SI["delta_so"]))
    assert np.abs(np.linalg.eigvalsh(H) - np.sort(ref)).max() < 1e-12


def test_hard_wall_box_separable_limit():
    """g2 = g3 = 0: E = g1 E0 sum_a lambda_{n_a}, fourfold (Gamma8) and
    twofold (+Delta, Gamma7)."""
    m = dict(SI, gamma2=0.0, gamma3=0.0)
    g = Grid(4, 3, 5, 0.5)
    H = hamiltonian_ls(g, m).toarray()
    lam = [(2 - 2 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1))) / g.h**2
           for n in g.shape]
    s = (lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :]).ravel()
    base = E0 * m["gamma1"] * s
    ref = np.sort(np.concatenate([np.repeat(base, 4), np.repeat(base + m["delta_so"], 2)]))
    assert np.abs(np.linalg.eigvalsh(H) - ref).max() < 1e-12


def test_harmonic_limit_richardson():
    """g2 = g3 = 0 chain along z in the oscillator well of the recipe:
    levels -> hbar w (n + 1/2) after removing the transverse hard-wall constant,
    O(h^2) error removed by Richardson extrapolation."""
    m = dict(SI, gamma2=0.0, gamma3=0.0)
    hw = 0.002
    Lbox = 160.0
    levels = {}
    for h in (1.0, 0.5):
        nz = int(round(Lbox / h)) - 1
        g = Grid(1, 1, nz, h)
        _, _, z = g.coords()
        V = hw**2 * (z - g.centre()[2]) ** 2 / (4 * m["gamma1"] * E0)
        H = hamiltonian_ls(g, m, V.ravel())
        w = sla.eigh(H.toarray(), eigvals_only=True, subset_by_index=(0, 11))
        levels[h] = w - E0 * m["gamma1"] * 4.0 / h**2
    rich = (4 * levels[0.5] - levels[1.0]) / 3.0
    ref = np.repeat(hw * (np.arange(3) + 0.5), 4)
    assert np.abs(rich - ref).max() < 1e-6
    assert np.abs(levels[0.5] - ref).max() > 1e-7   # the extrapolation did work


# ----------------------------------------------------------------------------
# symmetries of the magnetic terms
# ----------------------------------------------------------------------------

def _spectrum(g, V, e, B, gauge="symmetric", k=None):
    H = hamiltonian_ls(g, SI, V, e, B, gauge=gauge).toarray()
    w = np.linalg.eigvalsh(H)
    return w if k is None else w[:k]


def test_kramers_degeneracy_at_zero_field():
    g = Grid(4, 4, 3, 0.5)
    V, e = _random_fields(g, 5)
    w = _spectrum(g, V, e, (0, 0, 0))
    assert np.abs(w[0::2] - w[1::2]).max() < 1e-12
    assert np.diff(w[0::2]).min() > 1e-9        # pairs, not higher multiplets


def test_time_reversal_and_gauge_invariance():
    g = Grid(4, 3, 4, 0.5)
    V, e = _random_fields(g, 6)
    B = (1.3, -0.8, 2.1)
    w = _spectrum(g, V, e, B)
    wm = _spectrum(g, V, e, tuple(-b for b in B))
    wl = _spectrum(g, V, e, B, gauge="landau")
    assert np.abs(w - wm).max() < 1e-12
    assert np.abs(w - wl).max() < 1e-12
    assert np.abs(w[0::2] - w[1::2]).max() > 1e-6    # Kramers pairs are split


def test_linear_zeeman_first_order():
    """E(B) - E(0) = eigenvalues of dH/dB projected on each Kramers pair, up to O(B^2)."""
    g = Grid(4, 3, 4, 0.5)
    V, e = _random_fields(g, 7)
    direction = np.array([0.3, -0.5, 0.81])
    H0 = hamiltonian_ls(g, SI, V, e).toarray()
    w0, v0 = np.linalg.eigh(H0)
    errs = []
    for b in (0.02, 0.01):
        Hb = hamiltonian_ls(g, SI, V, e, tuple(b * direction)).toarray()
        wb = np.linalg.eigvalsh(Hb)
        dH = Hb - H0
        err = 0.0
        for p in range(3):
            P = v0[:, 2 * p:2 * p + 2]
            first = np.linalg.eigvalsh(P.conj().T @ dH @ P)
            err = max(err, np.abs(wb[2 * p:2 * p + 2] - w0[2 * p:2 * p + 2] - first).max())
        errs.append(err)
    assert errs[1] < 1e-8
    assert 3.0 < errs[0] / errs[1] < 5.0          # quadratic remainder


def test_onsite_zeeman_closed_form_mj_sectors():
    """B along z: m_j = +-3/2 at +-3 kappa mu_B B; the m_j = +-1/2 sectors are
    2x2 problems mixing Gamma8 and Gamma7 (written in the (m_l, m_s) basis)."""
    kap, D = SI["kappa"], SI["delta_so"]
    for Bz in (0.5, 3.0, 40.0):
        z = MU_B * Bz
        blocks = [np.array([[D / 3 + z, -np.sqrt(2) * D / 3],
                            [-np.sqrt(2) * D / 3, 2 * D / 3 + z * (3 * kap - 2)]]),
                  np.array([[D / 3 - z, -np.sqrt(2) * D / 3],
                            [-np.sqrt(2) * D / 3, 2 * D / 3 + z * (2 - 3 * kap)]])]
        ref = [3 * kap * z, -3 * kap * z]
        for b in blocks:
            ref.extend(np.linalg.eigvalsh(b))
        got = np.linalg.eigvalsh(onsite_so_zeeman_ls(SI, (0, 0, Bz)))
        assert np.abs(got - np.sort(ref)).max() < 1e-15
        # rotational invariance: same spectrum for any direction
        d = np.array([1.0, -2.0, 0.5])
        d = d / np.linalg.norm(d)
        got2 = np.linalg.eigvalsh(onsite_so_zeeman_ls(SI, tuple(Bz * d)))
        assert np.abs(got2 - np.sort(ref)).max() < 1e-14


def test_zeeman_projects_to_2kappa_muB_J_on_gamma8():
    """Wigner-Eckart: on Gamma8 the Zeeman term is 2 kappa mu_B B.J; in the
    |J m_j> basis with B along z the Gamma8 block is diagonal in m_j."""
    Bz = 0.1
    hz = onsite_so_zeeman_ls(SI, (0, 0, Bz)) - onsite_so_zeeman_ls(SI)
    hj = U_J_FROM_LS @ hz @ U_J_FROM_LS.conj().T
    ref = 2 * SI["kappa"] * MU_B * Bz * np.diag([1.5, 0.5, -0.5, -1.5])
    assert np.abs(hj[:4, :4] - ref).max() < 1e-18
    # Gamma7 block: (2 kappa - 1) mu_B B sigma_z
    ref7 = (2 * SI["kappa"] - 1) * MU_B * Bz * np.diag([1.0, -1.0])
    assert np.abs(hj[4:, 4:] - ref7).max() < 1e-18


# ----------------------------------------------------------------------------
# solvers and the adjoint
# ----------------------------------------------------------------------------

def test_arpack_matches_dense_on_harmonic_workload():
    from synth import workload
    w = workload("harmonic_10x8x8")
    g = Grid(w.nx, w.ny, w.nz, w.h)
    H = hamiltonian_ls(g, SI, w.V)
    Ed, _ = lowest_dense(H, w.nev)
    Ea, va = lowest_arpack(H, w.nev, tol=1e-14)
    assert np.abs(Ed - Ea).max() < 1e-10
    r = np.linalg.norm(H @ va - va * Ea, axis=0)
    assert r.max() < 1e-9


def test_hellmann_feynman_vs_central_differences():
    g = Grid(6, 4, 4, 0.5)
    r = np.random.default_rng(8)
    V_bg = 0.01 * r.standard_normal(g.npts)
    L = 0.2 * r.random((3, g.npts))
    e = 1e-3 * r.standard_normal((g.npts, 6))
    nev = 4

    def esum(vg):
        H = hamiltonian_ls(g, SI, gate_potential(V_bg, L, vg), e)
        return lowest_dense(H, nev)[0].sum()

    vg0 = np.array([0.01, -0.02, 0.005])
    H = hamiltonian_ls(g, SI, gate_potential(V_bg, L, vg0), e)
    E, v = lowest_dense(H, nev)
    grad = hf_gradient(v, np.ones(nev), L)
    d = 1e-4
    fd = np.array([(esum(vg0 + d * np.eye(3)[k]) - esum(vg0 - d * np.eye(3)[k])) / (2 * d)
                   for k in range(3)])
    assert np.abs(grad - fd).max() <= 1e-6 * np.abs(fd).max()
