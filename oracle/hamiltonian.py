"""Assembly of the single-particle hole Hamiltonian H_NI = H_LK + H_PB + V
(paper Eq. HNI), in two independent forms.

Hole picture: H = -H_valence, so confined hole states are the LOWEST
eigenvalues (the paper's "highest" hole states before the sign flip).

Form 1 -- |L S> basis (paper Eq. LK and the basis listed after it):
    order |X up>,|Y up>,|Z up>,|X dn>,|Y dn>,|Z dn>  (spin-major, c = 3 s + o)
    H = E0 (I_spin (x) H_kin) + H_so + H_Z + I_spin (x) H_eps(r) + V(r)
    H_kin (orbital 3x3 of operators), L = g1+4g2, M = g1-2g2, N = 6 g3:
        (H_kin)_ii = L K_ii + M sum_{a != i} K_aa,   (H_kin)_ij = N Ksym_ij
    H_so = (Delta/3) (I - sum_a sigma_a (x) L_a),  (L_a)_bc = -i eps_abc
           -> Gamma8 at 0, Gamma7 at +Delta
    H_Z  = mu_B sum_a B_a [(3 kappa - 1) I (x) L_a + sigma_a (x) I]
           (projects to 2 kappa mu_B B.J on Gamma8; q = 0)
    H_eps (Bir-Pikus, orbital): (H_eps)_ii = l e_ii + m (tr e - e_ii),
           (H_eps)_ij = n e_ij,  l = -(a_v + 2b), m = -(a_v - b), n = -sqrt(3) d

Form 2 -- |J m_j> basis in the order the paper lists (Sec. II.C):
    |3/2,+3/2>,|3/2,+1/2>,|3/2,-1/2>,|3/2,-3/2>,|1/2,+1/2>,|1/2,-1/2>
    the standard 6x6 Luttinger-Kohn matrix built from P, Q, R, S (units E0)
        P = g1 k^2, Q = g2 (kx^2+ky^2-2kz^2),
        R = sqrt3 [-g2 (kx^2-ky^2) + 2i g3 kx ky], S = 2 sqrt3 g3 (kx - i ky) kz
    with k_a^2 -> K_aa and k_a k_b -> Ksym_ab; strain by the Bir-Pikus
    substitution P_e = -a_v tr e, Q_e = -(b/2)(exx+eyy-2ezz),
    R_e = (sqrt3/2) b (exx-eyy) - i d exy, S_e = -d (exz - i eyz);
    spin-orbit Delta on the two |1/2> states; Zeeman rotated from Form 1.

Strain input is the symmetric tensor in Voigt order (xx, yy, zz, yz, xz, xy),
tensor (not engineering) shear components.

Row index of the assembled matrix: p * 6 + c  (grid point slow, component fast).
"""

import numpy as np
import scipy.sparse as sp

from .constants import E0, MU_B
from .grid import kinetic_operators

_S3 = np.sqrt(3.0)
_S2 = np.sqrt(2.0)

# psi_J = U psi_LS for each grid point.  Rows: |J m_j> in the paper's order,
# columns: |L S> in the paper's order.  The defining property (checked by the
# tests) is U H_LS U^H = H_J for every wavevector, strain and field.
U_J_FROM_LS = np.array([
    [1j * _S3, _S3, 0, 0, 0, 0],
    [0, 0, -2j, 1j, 1, 0],
    [-1j, 1, 0, 0, 0, -2j],
    [0, 0, 0, -1j * _S3, _S3, 0],
    [0, 0, -1j * _S2, -1j * _S2, -_S2, 0],
    [-1j * _S2, _S2, 0, 0, 0, 1j * _S2],
], dtype=complex) / np.sqrt(6.0)

# Pauli matrices and the orbital angular momentum on (X, Y, Z)
_SIG = [np.array([[0, 1], [1, 0]], dtype=complex),
        np.array([[0, -1j], [1j, 0]], dtype=complex),
        np.array([[1, 0], [0, -1]], dtype=complex)]


def _levi_civita():
    e = np.zeros((3, 3, 3))
    e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1.0
    e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1.0
    return e


_LORB = [-1j * _levi_civita()[a] for a in range(3)]


def _mat(m):
    out = dict(m)
    return out


def onsite_so_zeeman_ls(material, B=(0.0, 0.0, 0.0)):
    """Constant 6x6 spin-orbit + Zeeman matrix in the |L S> basis."""
    d = material["delta_so"]
    kap = material["kappa"]
    I2 = np.eye(2)
    I3 = np.eye(3)
    hso = np.eye(6, dtype=complex)
    for a in range(3):
        hso = hso - np.kron(_SIG[a], _LORB[a])
    hso = hso * (d / 3.0)
    hz = np.zeros((6, 6), dtype=complex)
    for a in range(3):
        hz = hz + float(B[a]) * ((3.0 * kap - 1.0) * np.kron(I2, _LORB[a])
                                 + np.kron(_SIG[a], I3))
    return hso + MU_B * hz


def strain_orbital_ls(material, strain):
    """Per-point orbital Bir-Pikus matrix (..., 3, 3) from Voigt strain (..., 6)."""
    av, b, dd = material["a_v"], material["b"], material["d"]
    l_ = -(av + 2.0 * b)
    m_ = -(av - b)
    n_ = -np.sqrt(3.0) * dd
    e = np.asarray(strain, dtype=float)
    tr = e[..., 0] + e[..., 1] + e[..., 2]
    out = np.zeros(e.shape[:-1] + (3, 3))
    for i in range(3):
        out[..., i, i] = l_ * e[..., i] + m_ * (tr - e[..., i])
    # Voigt: 3 -> yz, 4 -> xz, 5 -> xy
    for (i, j, v) in ((1, 2, 3), (0, 2, 4), (0, 1, 5)):
        out[..., i, j] = n_ * e[..., v]
        out[..., j, i] = n_ * e[..., v]
    return out


def _unit(n, i, j):
    m = np.zeros((n, n), dtype=complex)
    m[i, j] = 1.0
    return m


def _check_fields(grid, V, strain):
    N = grid.npts
    V = np.zeros(N) if V is None else np.asarray(V, dtype=float).reshape(N)
    if strain is not None:
        strain = np.asarray(strain, dtype=float).reshape(N, 6)
    return V, strain


def hamiltonian_ls(grid, material, V=None, strain=None, B=(0.0, 0.0, 0.0),
                   gauge="symmetric"):
    """Sparse (6N x 6N) Hamiltonian in the |L S> basis (Form 1 above)."""
    g1, g2, g3 = material["gamma1"], material["gamma2"], material["gamma3"]
    V, strain = _check_fields(grid, V, strain)
    N = grid.npts
    Kaa, _, Ksym = kinetic_operators(grid, B, gauge)
    L_, M_, N_ = g1 + 4.0 * g2, g1 - 2.0 * g2, 6.0 * g3
    I2 = np.eye(2)
    terms = []
    for o in range(3):
        op = L_ * Kaa[o]
        for a in range(3):
            if a != o:
                op = op + M_ * Kaa[a]
        terms.append(sp.kron(E0 * op, np.kron(I2, _unit(3, o, o)), format="csr"))
    for o in range(3):
        for o2 in range(3):
            if o != o2:
                terms.append(sp.kron(E0 * N_ * Ksym[(o, o2)],
                                     np.kron(I2, _unit(3, o, o2)), format="csr"))
    if strain is not None:
        D = strain_orbital_ls(material, strain)
        for o in range(3):
            for o2 in range(3):
                dv = D[:, o, o2]
                if np.any(dv != 0.0):
                    terms.append(sp.kron(sp.diags(dv), np.kron(I2, _unit(3, o, o2)),
                                         format="csr"))
    terms.append(sp.kron(sp.diags(V), np.eye(6), format="csr"))
    terms.append(sp.kron(sp.identity(N), onsite_so_zeeman_ls(material, B), format="csr"))
    H = terms[0]
    for t in terms[1:]:
        H = H + t
    return H.tocsr()


def _chuang_pattern(P, Q, R, S):
    """6x6 block pattern of the Luttinger-Kohn matrix from operator blocks.

    Returns a dict {(row, col): sparse operator}.  P and Q are Hermitian;
    R^H and S^H denote operator adjoints.
    """
    Rh = R.getH()
    Sh = S.getH()
    r2 = _S2
    r32 = np.sqrt(1.5)
    blocks = {
        (0, 0): P + Q, (0, 1): -S, (0, 2): R, (0, 4): -S / r2, (0, 5): r2 * R,
        (1, 0): -Sh, (1, 1): P - Q, (1, 3): R, (1, 4): -r2 * Q, (1, 5): r32 * S,
        (2, 0): Rh, (2, 2): P - Q, (2, 3): S, (2, 4): r32 * Sh, (2, 5): r2 * Q,
        (3, 1): Rh, (3, 2): Sh, (3, 3): P + Q, (3, 4): -r2 * Rh, (3, 5): -Sh / r2,
        (4, 0): -Sh / r2, (4, 1): -r2 * Q, (4, 2): r32 * S, (4, 3): -r2 * R, (4, 4): P,
        (5, 0): r2 * Rh, (5, 1): r32 * Sh, (5, 2): r2 * Q, (5, 3): -S / r2, (5, 5): P,
    }
    return blocks


def _assemble(blocks, N):
    H = None
    for (i, j), op in blocks.items():
        t = sp.kron(op, _unit(6, i, j), format="csr")
        H = t if H is None else H + t
    return H


def hamiltonian_j(grid, material, V=None, strain=None, B=(0.0, 0.0, 0.0),
                  gauge="symmetric", origin=None):
    """Sparse (6N x 6N) Hamiltonian in the |J m_j> basis (Form 2 above); origin: the
    symmetric gauge's origin as an offset from the box centre (nm), None for the centre."""
    g1, g2, g3 = material["gamma1"], material["gamma2"], material["gamma3"]
    V, strain = _check_fields(grid, V, strain)
    N = grid.npts
    Kaa, _, Ksym = kinetic_operators(grid, B, gauge, origin)
    P = g1 * (Kaa[0] + Kaa[1] + Kaa[2])
    Q = g2 * (Kaa[0] + Kaa[1] - 2.0 * Kaa[2])
    R = _S3 * (-g2 * (Kaa[0] - Kaa[1]) + 2j * g3 * Ksym[(0, 1)])
    S = 2.0 * _S3 * g3 * (Ksym[(0, 2)] - 1j * Ksym[(1, 2)])
    H = _assemble(_chuang_pattern(E0 * P, E0 * Q, E0 * R, E0 * S), N)
    if strain is not None:
        av, b, dd = material["a_v"], material["b"], material["d"]
        e = strain
        Pe = sp.diags(-av * (e[:, 0] + e[:, 1] + e[:, 2])).astype(complex)
        Qe = sp.diags(-(b / 2.0) * (e[:, 0] + e[:, 1] - 2.0 * e[:, 2])).astype(complex)
        Re = sp.diags((_S3 / 2.0) * b * (e[:, 0] - e[:, 1]) - 1j * dd * e[:, 5])
        Se = sp.diags(-dd * (e[:, 4] - 1j * e[:, 3]))
        H = H + _assemble(_chuang_pattern(Pe.tocsr(), Qe.tocsr(), Re.tocsr(), Se.tocsr()), N)
    so = np.diag([0, 0, 0, 0, material["delta_so"], material["delta_so"]]).astype(complex)
    # Zeeman: the |L S> form rotated into this basis (the paper prints none)
    hz_ls = onsite_so_zeeman_ls(material, B) - onsite_so_zeeman_ls(material, (0.0, 0.0, 0.0))
    hz_j = U_J_FROM_LS @ hz_ls @ U_J_FROM_LS.conj().T
    H = H + sp.kron(sp.diags(V), np.eye(6), format="csr")
    H = H + sp.kron(sp.identity(N), so + hz_j, format="csr")
    return H.tocsr()


def to_j_basis(psi_ls):
    """Map eigenvectors (6N, k) from |L S> to |J m_j> component order."""
    psi = np.asarray(psi_ls)
    k = psi.shape[1] if psi.ndim == 2 else 1
    p = psi.reshape(-1, 6, k)
    out = np.einsum("jc,nck->njk", U_J_FROM_LS, p)
    return out.reshape(psi.shape)
