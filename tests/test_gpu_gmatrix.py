"""GPU parity of the double dot's g-matrices and of the effective two-spin model
(Sec. III: Eqs. HB, J_QD, J_anis) against the CPU oracle, through the C ABI.

The GPU forms dH/dB from one B = 0 stencil apply to the position-weighted states
and one Gram product; the oracle differentiates H(B) numerically.  Bars: the
g-matrices of the bonding and antibonding doublets (the same doublet bases on
both sides) within 1e-8 of the oracle's, relative; the dots' symmetric g-tensors
(basis-free) and centres likewise; the effective model's fields, spectrum and
exchange components within 1e-12 relative on the same g-tensors.  At full size:
time reversal, mirror structure where it holds, and the Zeeman splitting of GPU
solves at small B.
"""

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid
from oracle.constants import MU_B
from oracle.gmatrix import double_dot_g, two_spin_model
from synth import workload

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a))


def _mirror_dqd(shape, h):
    nx, ny, nz = shape
    x = (np.arange(nx) - 0.5 * (nx - 1)) * h
    y = (np.arange(ny) - 0.5 * (ny - 1)) * h
    z = (np.arange(nz) - 0.5 * (nz - 1)) * h
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    x0 = 0.25 * nx * h
    return 0.08 * (np.abs(X) < 0.12 * nx * h) + 0.004 * (np.abs(X) - x0) ** 2 + \
        0.01 * (Y ** 2 + 0.7 * Z ** 2)


def _states(V, h, strain):
    import paper_2607_08447_amd as hkp
    r = hkp.solve(_t(V), h, 4, strain=_t(strain), tol=1e-11, precision="fp64")
    assert r.status == 0
    return r


def _vs_oracle(V, h, strain):
    import paper_2607_08447_amd as hkp
    r = _states(V, h, strain)
    gm = hkp.g_matrices(r.psi, _t(V), h, strain=_t(strain))
    grid = Grid(*V.shape, h)
    psi = r.psi.cpu().numpy().reshape(4, -1).T
    ref = double_dot_g(grid, SI_MATERIAL, psi, r.E.cpu().numpy(), V.ravel(),
                       None if strain is None else strain.reshape(-1, 6))
    scale = max(np.abs(ref["g"][0]).max(), np.abs(ref["g"][1]).max())
    err = max(np.abs(gm.g_sym[k] - ref["g_sym"][k]).max() for k in range(4)) / scale
    print(f"largest g_sym difference {err:.2e} (relative)", flush=True)
    for k in (0, 1):   # the input states' own bases: g itself agrees
        assert np.abs(gm.g[k] - ref["g"][k]).max() <= 1e-8 * scale, k
    for k in range(4):
        assert np.abs(gm.g_sym[k] - ref["g_sym"][k]).max() <= 1e-8 * scale, k
        assert np.abs(np.linalg.svd(gm.g[k], compute_uv=False) -
                      np.linalg.svd(ref["g"][k], compute_uv=False)).max() <= 1e-8 * scale
        assert np.abs(gm.centre[k] - ref["centre"][k]).max() <= 1e-9
    assert np.abs(gm.kramers[:2]).max() <= 1e-7 * scale
    assert abs(gm.delta - ref["delta"]) <= 1e-10 and abs(gm.t - ref["t"]) <= 1e-10
    assert abs(gm.d - ref["d"]) <= 1e-9
    assert np.abs(gm.E - r.E.cpu().numpy()).max() <= 1e-10
    return gm, ref


def test_g_matrices_vs_oracle_dqd_small():
    w = workload("dqd_small")
    print("g-matrices dqd_small", flush=True)
    _vs_oracle(w.V, w.h, w.strain)


def test_g_matrices_mirror_symmetric_double_dot():
    """No strain, V(-x) = V(x): mirror-image dots, g_R = P g_L P, P = diag(1, -1, -1)."""
    V = _mirror_dqd((32, 8, 8), 0.5)
    print("g-matrices mirror dqd 32x8x8", flush=True)
    gm, _ = _vs_oracle(V, 0.5, None)
    P = np.diag([1.0, -1.0, -1.0])
    s = np.abs(gm.g_sym[2]).max()
    assert np.abs(gm.g_sym[3] - P @ gm.g_sym[2] @ P).max() <= 1e-7 * s
    assert gm.centre[2][0] < 0 < gm.centre[3][0]
    assert abs(gm.centre[2][0] + gm.centre[3][0]) <= 1e-7


def test_two_spin_model_vs_oracle():
    import torch
    import paper_2607_08447_amd as hkp
    w = workload("dqd_small")
    r = _states(w.V, w.h, w.strain)
    gm = hkp.g_matrices(r.psi, _t(w.V), w.h, strain=_t(w.strain))
    rng = np.random.default_rng(3)
    B = rng.normal(size=(257, 3)) * np.exp(rng.uniform(-5, 0, size=(257, 1)))
    B[0] = 0.0
    B[1] = (0.0, 0.0, 0.05)
    J, n_so, lam = 2.3e-7, (0.3, -1.0, 0.2), 45.0
    out = hkp.two_spin_model(gm, J, torch.from_numpy(B), n_so, lam, return_matrix=True)
    theta = gm.d / lam
    for k in range(1, len(B)):
        ref = two_spin_model(gm.g_sym[2], gm.g_sym[3], gm.t, J, theta, n_so, B[k])
        sb = np.abs(ref["bbar"]).max() + np.abs(ref["db"]).max()
        assert np.abs(out["bbar"][k].cpu().numpy() - ref["bbar"]).max() <= 1e-12 * sb
        assert np.abs(out["db"][k].cpu().numpy() - ref["db"]).max() <= 1e-12 * sb
        assert abs(float(out["dEz"][k]) - ref["dEz"]) <= 1e-12 * sb
        Hs = np.abs(ref["H"]).max()
        assert np.abs(out["H"][k].cpu().numpy() - ref["H"]).max() <= 1e-14 * Hs
        assert np.abs(out["E"][k].cpu().numpy() - ref["E"]).max() <= 1e-13 * Hs
        assert np.abs(out["Jt"][k].cpu().numpy() - ref["Jt"]).max() <= 1e-12 * J
        assert abs(float(out["J_perp"][k]) - ref["J_perp"]) <= 1e-12 * J
        assert abs(float(out["J_par"][k]) - ref["J_par"]) <= 1e-12 * J
    # B = 0: the lab frames, no Zeeman fields, the singlet pair and a triple zero
    assert float(out["dEz"][0]) == 0.0 and np.abs(out["bbar"][0].cpu().numpy()).max() == 0.0
    E0 = np.sort(out["E"][0].cpu().numpy())
    Ue = 2 * gm.t ** 2 / J
    rr = np.sqrt(Ue * Ue / 4 + 2 * gm.t ** 2)
    assert np.abs(E0 - np.sort([Ue / 2 - rr, 0, 0, 0, Ue / 2 + rr])).max() <= 1e-13 * Ue


def test_two_spin_model_rejects_bad_options():
    import torch
    import paper_2607_08447_amd as hkp
    from paper_2607_08447_amd._lib import HkpError
    gm = torch.zeros(103, dtype=torch.float64, device="cuda")
    with pytest.raises(HkpError):
        hkp.two_spin_model(gm, 1e-7, torch.zeros(4, 3), (0, 0, 0), 10.0)
    with pytest.raises(HkpError):
        hkp.two_spin_model(gm, 1e-7, torch.zeros(4, 3), (0, 0, 1), 0.0)


def test_g_matrices_full_size_zeeman_splitting():
    """256 x 48 x 48 double dot with strain: the bonding doublet's g-matrix gives the
    splitting of the lowest doublet in GPU solves at small B (first order, Richardson
    in |B|), for three field directions; time reversal on both eigen-doublets."""
    import paper_2607_08447_amd as hkp
    w = workload("dqd_256x48x48")
    print("g-matrices dqd_256x48x48", flush=True)
    r = hkp.solve(_t(w.V), w.h, 4, strain=_t(w.strain), tol=1e-10, precision="fp64")
    assert r.status == 0
    gm = hkp.g_matrices(r.psi, _t(w.V), w.h, strain=_t(w.strain))
    s = np.abs(gm.g[0]).max()
    assert np.abs(gm.kramers[:2]).max() <= 1e-6 * s
    assert gm.delta > 0
    rng = np.random.default_rng(1)
    beta = 2e-3 * gm.delta / (MU_B * s)   # Zeeman energy 1e-3 of the doublet splitting
    for _ in range(3):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        sl = []
        for b in (beta, 2 * beta):
            rb = hkp.solve(_t(w.V), w.h, 4, strain=_t(w.strain), B=tuple(b * n), tol=1e-10,
                           precision="fp64")
            assert rb.status == 0
            E = rb.E.cpu().numpy()
            sl.append((E[1] - E[0]) / b)
        slope = (4 * sl[0] - sl[1]) / 3
        expect = MU_B * np.linalg.norm(gm.g[0] @ n)
        print(f"splitting slope {slope:.6e} vs mu_B |g n| {expect:.6e}", flush=True)
        assert abs(slope - expect) <= 1e-4 * expect
