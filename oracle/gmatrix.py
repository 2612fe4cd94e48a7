"""g-matrices of Kramers doublets and the effective two-spin model of the double
dot -- TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

Sec. III (two-qubit gates) builds the dots' g-tensors from the g-matrix of the
spin-mixed bonding and antibonding single-particle states, estimates the tunnel
coupling from their splitting, t = Delta / sqrt(2), and U - eps from the CI
exchange through J = 2 t^2 / (U - eps).  The g-tensors enter the 5 x 5 effective
Hamiltonian in the S(0,2), S(1,1), T+, T-, T0 basis (Eq. HB), and the exchange
matrix J R(-2 theta_so), seen in the two qubits' frames (Eq. J_QD), gives the
transverse and longitudinal exchange (Eqs. J_anis).  Readings taken here:

  * g-matrix of a Kramers doublet {u1, u2}: to first order in B the Hamiltonian
    restricted to the doublet is (mu_B / 2) sum_ab sigma_a g_ab B_b, so
    g_ab = Re tr(sigma_a M_b) / mu_B with M_b = <u_i| dH/dB_b |u_j> (2 x 2); g
    depends on the doublet basis only through a rotation on the left;
  * dH/dB_b is the derivative of the whole Hamiltonian (Zeeman and Peierls
    terms) at B = 0, in the symmetric gauge about the doublet's own centre of
    charge (the g-matrix of an exact eigen-doublet does not depend on the origin);
    here it is taken from its definition, by Richardson-extrapolated central
    differences of H(B);
  * the dots' doublets: the eigenvectors of the position x (the channel axis)
    within the span of the bonding and antibonding doublets, lower x = left;
  * symmetric g-tensor: sgn(det g) (g^T g)^(1/2), which a proper rotation of the
    doublet basis reaches from g;
  * R(theta) is the rotation by theta about n_so, theta_so = d / lambda_so;
    b_bar = mu_B (R(-theta_so) g_L + R(theta_so) g_R) B / 2,
    delta_b = mu_B (R(-theta_so) g_L - R(theta_so) g_R) B / 2, delta E_Z = |delta_b|;
  * the qubit frames: R_L n_L = z with n_L = g_L B / |g_L B| (the rotation about
    n_L x z; the remaining freedom about z leaves J_perp and J_par unchanged);
    J~ = R_L J R(-2 theta_so) R_R^T, J_perp and J_par as in Eqs. J_anis.
"""

import numpy as np

from .constants import E_OVER_HBAR, MU_B  # noqa: F401  (E_OVER_HBAR: units of the gauge)
from .hamiltonian import hamiltonian_j

SIGMA = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]


def field_derivative(grid, material, V=None, strain=None, origin=None, step=1e-2):
    """dH/dB_b at B = 0 (b = x, y, z), |J m_j> basis, symmetric gauge about origin.

    Central differences at s and 2s combined to cancel the s^2 term:
    [8 (H(s) - H(-s)) - (H(2s) - H(-2s))] / (12 s).  The Zeeman part is linear in
    B and comes out exactly; a Peierls factor exp(i theta B) keeps an error of
    order (theta s)^4 relative."""
    out = []
    for b in range(3):
        e = np.zeros(3)
        e[b] = 1.0

        def H(s):
            return hamiltonian_j(grid, material, V, strain, B=tuple(s * e), origin=origin)

        d1 = H(step) - H(-step)
        d2 = H(2 * step) - H(-2 * step)
        out.append(((8.0 * d1 - d2) / (12.0 * step)).tocsr())
    return out


def positions(grid):
    """Coordinates about the box centre, each (N,) in the oracle's point order."""
    x, y, z = grid.coords()
    c = grid.centre()
    return [(x - c[0]).ravel(), (y - c[1]).ravel(), (z - c[2]).ravel()]


def position_matrix(grid, psi, axis):
    """<psi_i| r_axis |psi_j> for psi (6N, k) with r about the box centre."""
    r = np.repeat(positions(grid)[axis], 6)
    return psi.conj().T @ (r[:, None] * psi)


def centre_of_charge(grid, psi2):
    """Mean position (nm, about the box centre) of the two states of a doublet."""
    return np.array([np.trace(position_matrix(grid, psi2, a)).real / psi2.shape[1]
                     for a in range(3)])


def g_matrix(psi2, D):
    """g_ab = Re tr(sigma_a M_b) / mu_B with M_b = psi2^H D_b psi2 (3 x 3, row a = Pauli)."""
    g = np.zeros((3, 3))
    for b in range(3):
        M = psi2.conj().T @ (D[b] @ psi2)
        for a in range(3):
            g[a, b] = np.trace(SIGMA[a] @ M).real / MU_B
    return g


def zeeman_trace(psi2, D):
    """tr M_b / mu_B: zero for a Kramers doublet (the field derivative is odd under time reversal)."""
    return np.array([np.trace(psi2.conj().T @ (D[b] @ psi2)).real / MU_B for b in range(3)])


def symmetric_g(g):
    """sgn(det g) (g^T g)^(1/2)."""
    w, Q = np.linalg.eigh(g.T @ g)
    s = -1.0 if np.linalg.det(g) < 0 else 1.0
    return s * (Q * np.sqrt(np.clip(w, 0.0, None))) @ Q.T


def localise(grid, psi4):
    """The left and right doublets: eigenvectors of x within span(psi4), ascending."""
    X = position_matrix(grid, psi4, 0)
    X = 0.5 * (X + X.conj().T)
    _, C = np.linalg.eigh(X)
    return psi4 @ C[:, :2], psi4 @ C[:, 2:]


def doublet_g(grid, material, psi2, V=None, strain=None):
    """g-matrix of one doublet, dH/dB in the symmetric gauge about its centre of charge."""
    r0 = centre_of_charge(grid, psi2)
    D = field_derivative(grid, material, V, strain, origin=r0)
    return g_matrix(psi2, D), r0, zeeman_trace(psi2, D)


def double_dot_g(grid, material, psi4, E4, V=None, strain=None):
    """The four g-matrices (bonding, antibonding, left, right), their doublets'
    centres, Delta and t, from the two lowest Kramers doublets psi4 (6N, 4) at B = 0."""
    left, right = localise(grid, psi4)
    out = {"g": [], "centre": [], "trace": []}
    for psi2 in (psi4[:, :2], psi4[:, 2:], left, right):
        g, r0, tr = doublet_g(grid, material, psi2, V, strain)
        out["g"].append(g)
        out["centre"].append(r0)
        out["trace"].append(tr)
    out["g_sym"] = [symmetric_g(g) for g in out["g"]]
    E4 = np.asarray(E4, dtype=float)
    out["delta"] = 0.5 * (E4[2] + E4[3]) - 0.5 * (E4[0] + E4[1])
    out["t"] = tunnel_coupling(out["delta"])
    out["d"] = float(np.linalg.norm(out["centre"][3] - out["centre"][2]))
    return out


def tunnel_coupling(delta):
    """t = Delta / sqrt(2) from the bonding-antibonding splitting at zero detuning."""
    return abs(delta) / np.sqrt(2.0)


def u_minus_eps(t, J):
    """U - eps from J = 2 t^2 / (U - eps)."""
    return 2.0 * t * t / J


def rotation(n, angle):
    """Rotation by angle about the unit vector along n (right-hand rule)."""
    n = np.asarray(n, dtype=float)
    n = n / np.linalg.norm(n)
    K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def zeeman_fields(gL, gR, theta, n_so, B):
    """b_bar and delta_b (eV) of the effective model."""
    B = np.asarray(B, dtype=float)
    a = rotation(n_so, -theta) @ gL @ B
    b = rotation(n_so, theta) @ gR @ B
    return MU_B * (a + b) / 2.0, MU_B * (a - b) / 2.0


def effective_hamiltonian(U_eps, t, bbar, db):
    """Eq. HB in the basis S(0,2), S(1,1), T+, T-, T0."""
    r2 = np.sqrt(2.0)
    bx, by, bz = bbar
    dx, dy, dz = db
    H = np.zeros((5, 5), dtype=complex)
    H[0, 0] = U_eps
    H[0, 1] = H[1, 0] = r2 * t
    H[1, 2] = -(dx + 1j * dy) / r2
    H[1, 3] = (dx - 1j * dy) / r2
    H[1, 4] = dz
    H[2, 2] = bz
    H[3, 3] = -bz
    H[2, 4] = (bx - 1j * by) / r2
    H[3, 4] = (bx + 1j * by) / r2
    for i, j in ((1, 2), (1, 3), (1, 4), (2, 4), (3, 4)):
        H[j, i] = np.conj(H[i, j])
    return H


def qubit_frame(n):
    """A proper rotation R with R n = z: the rotation about n x z by the angle between them."""
    n = np.asarray(n, dtype=float)
    n = n / np.linalg.norm(n)
    z = np.array([0.0, 0.0, 1.0])
    axis = np.cross(n, z)
    s, c = np.linalg.norm(axis), float(n @ z)
    if s < 1e-300:
        return np.eye(3) if c > 0 else np.diag([1.0, -1.0, -1.0])
    return rotation(axis, np.arctan2(s, c))


def exchange_components(Jt):
    """|J_perp| and J_par of the exchange matrix in the qubit frames (Eqs. J_anis)."""
    perp = 0.5 * np.hypot(Jt[0, 0] + Jt[1, 1], Jt[0, 1] - Jt[1, 0])
    return perp, Jt[2, 2]


def anisotropic_exchange(J, theta, n_so, gL, gR, B, RL=None, RR=None):
    """J_hat = J R(-2 theta), J~ = R_L J_hat R_R^T, and (|J_perp|, J_par)."""
    B = np.asarray(B, dtype=float)
    Jhat = J * rotation(n_so, -2.0 * theta)
    RL = qubit_frame(gL @ B) if RL is None else RL
    RR = qubit_frame(gR @ B) if RR is None else RR
    Jt = RL @ Jhat @ RR.T
    perp, par = exchange_components(Jt)
    return Jhat, Jt, perp, par


def two_spin_model(gL, gR, t, J, theta, n_so, B):
    """Everything the effective model gives for one field: b_bar, delta_b,
    delta E_Z, the spectrum of Eq. HB, J~, |J_perp|, J_par."""
    bbar, db = zeeman_fields(gL, gR, theta, n_so, B)
    H = effective_hamiltonian(u_minus_eps(t, J), t, bbar, db)
    _, Jt, perp, par = anisotropic_exchange(J, theta, n_so, gL, gR, B)
    return {"bbar": bbar, "db": db, "dEz": float(np.linalg.norm(db)), "H": H,
            "E": np.linalg.eigvalsh(H), "Jt": Jt, "J_perp": perp, "J_par": par}
