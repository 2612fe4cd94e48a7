"""Hellmann-Feynman backward: the GPU kernel against the oracle's gradient
formula, and the autograd path against central finite differences
(dV = 1e-4 V) at the relative tolerance 1e-5 of the workload definition."""

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid, gate_potential, hamiltonian_ls, hf_gradient, lowest_arpack

pytestmark = pytest.mark.gpu


def _small_adjoint():
    # the adjoint workload's recipe on a grid the oracle handles in seconds
    from synth.inputs import build
    ws = build("adjoint_dqd_192x40x40", small_shape=(72, 12, 10))
    return ws


def test_hf_kernel_matches_oracle_formula():
    import torch
    import paper_2607_08447_amd as hkp
    r = np.random.default_rng(3)
    shape = (20, 7, 5)
    N = int(np.prod(shape))
    nev, G = 6, 5
    psi = r.standard_normal((nev, N * 6)) + 1j * r.standard_normal((nev, N * 6))
    wts = r.random(nev)
    L = r.random((G, N))
    g = hkp.hf_grad(torch.from_numpy(psi.reshape((nev,) + shape + (6,))), torch.from_numpy(wts),
                    torch.from_numpy(L)).cpu().numpy()
    ref = hf_gradient(psi.T, wts, L)
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()


def test_autograd_vs_finite_differences_and_oracle():
    import torch
    import paper_2607_08447_amd as hkp
    w = _small_adjoint()
    Lg = w.extra["L"]
    nev = 8
    cfg = dict(h=w.h, nev=nev, strain=torch.from_numpy(w.strain), B=w.B, nb=16, tol=1e-10)
    Vg = torch.zeros(5, dtype=torch.float64, device="cuda", requires_grad=True)
    Ld = torch.from_numpy(Lg).cuda()
    Vbg = torch.from_numpy(w.V).cuda()
    E = hkp.EigvalsFromPotential.apply(Vg, Ld, Vbg, cfg)
    loss = E.sum()
    loss.backward()
    grad = Vg.grad.cpu().numpy()

    def esum(vg):
        V = Vbg + torch.tensordot(torch.as_tensor(vg, device="cuda"), Ld, dims=1)
        return float(hkp.solve(V, w.h, nev, strain=cfg["strain"], B=w.B, nb=16, tol=1e-10).E.sum())

    d = 1e-4
    fd = np.array([(esum(d * np.eye(5)[k]) - esum(-d * np.eye(5)[k])) / (2 * d) for k in range(5)])
    assert np.abs(grad - fd).max() <= 1e-5 * np.abs(fd).max(), (grad, fd)
    # oracle: Hellmann-Feynman from the oracle's own eigenvectors
    H = hamiltonian_ls(Grid(*w.shape, w.h), SI_MATERIAL,
                       gate_potential(w.V.ravel(), Lg.reshape(5, -1), np.zeros(5)),
                       w.strain.reshape(-1, 6), w.B)
    _, v = lowest_arpack(H, nev, tol=1e-13)
    ref = hf_gradient(v, np.ones(nev), Lg.reshape(5, -1))
    assert np.abs(grad - ref).max() <= 1e-7 * np.abs(ref).max()


def test_unequal_weights_in_kramers_pair_raise():
    import torch
    import paper_2607_08447_amd as hkp
    w = _small_adjoint()
    cfg = dict(h=w.h, nev=4, strain=torch.from_numpy(w.strain), B=w.B, nb=12, tol=1e-9)
    Vg = torch.zeros(5, dtype=torch.float64, device="cuda", requires_grad=True)
    E = hkp.EigvalsFromPotential.apply(Vg, torch.from_numpy(w.extra["L"]).cuda(),
                                       torch.from_numpy(w.V).cuda(), cfg)
    with pytest.raises(ValueError):
        E[0].backward()


def test_degenerate_tol_setting_reaches_the_backward():
    """cfg['degenerate_tol'] is a backward setting: the forward must not pass it
    to the solve, and the backward must use it to group degenerate levels."""
    import torch
    import paper_2607_08447_amd as hkp
    w = _small_adjoint()
    Ld = torch.from_numpy(w.extra["L"]).cuda()
    cfg = dict(h=w.h, nev=4, strain=torch.from_numpy(w.strain), B=w.B, nb=12, tol=1e-9,
               degenerate_tol=1e-7)
    Vg = torch.zeros(5, dtype=torch.float64, device="cuda", requires_grad=True)
    E = hkp.EigvalsFromPotential.apply(Vg, Ld, torch.from_numpy(w.V).cuda(), cfg)
    E.sum().backward()
    ref = hkp.hf_grad(hkp.solve(torch.from_numpy(w.V).cuda(), w.h, 4, strain=cfg["strain"],
                                B=w.B, nb=12, tol=1e-9).psi,
                      torch.ones(4, dtype=torch.float64, device="cuda"),
                      Ld.reshape(5, -1)).cpu().numpy()
    g = Vg.grad.cpu().numpy()
    assert np.abs(g - ref).max() <= 1e-7 * np.abs(ref).max()
    # the setting groups the Kramers pairs: unequal weights inside one still raise
    Vg1 = torch.zeros(5, dtype=torch.float64, device="cuda", requires_grad=True)
    E1 = hkp.EigvalsFromPotential.apply(Vg1, Ld, torch.from_numpy(w.V).cuda(), cfg)
    with pytest.raises(ValueError):
        E1[0].backward()
