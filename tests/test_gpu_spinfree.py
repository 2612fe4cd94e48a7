"""GPU parity of the spin-free single-particle basis (Eq. H0) and its spin-orbit
matrix (Eq. H1) against the CPU oracle, through the C ABI.

Bars: orbital energies within 1e-8 eV of the oracle's dense/ARPACK solve of the
orbital block (residual <= 1e-8 eV against the oracle's own matrix); the
spanned orbital subspace (projector) within 1e-6; the spin-orbit matrix of the
GPU's orbitals within 1e-12 of the oracle's formula on the same orbitals; the
spectrum of diag(E) + SOI (basis-invariant) within 1e-8 eV of the oracle's.
"""

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid, h0_orbital, single_particle, soi_matrix
from oracle.solve import lowest_arpack
from synth import workload

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a))


def _case(name):
    w = workload(name)
    return w, Grid(*w.shape, w.h)


@pytest.mark.parametrize("name,precision,bar", [("fin_small", "fp64", 1e-8),
                                                ("dqd_small", "fp64", 1e-8),
                                                ("dqd_small", "mixed", 1e-6)])
def test_spin_free_solve_vs_oracle(name, precision, bar):
    import paper_2607_08447_amd as hkp
    w, g = _case(name)
    nev = 12
    print(f"spin-free {name} {precision}", flush=True)
    tol = 1e-9 if precision == "fp64" else 1e-6
    r = hkp.solve(_t(w.V), w.h, nev, strain=_t(w.strain), nb=24, tol=tol, precision=precision,
                  spin_free=True)
    assert r.status == 0 and tuple(r.psi.shape) == (nev,) + w.shape + (3,)
    h0 = h0_orbital(g, SI_MATERIAL, V=w.V, strain=w.strain)
    E_ref, phi_ref = lowest_arpack(h0, nev + 1, tol=1e-14)
    E = r.E.cpu().numpy()
    assert np.abs(E - E_ref[:nev]).max() <= bar
    phi = r.psi.cpu().numpy().reshape(nev, -1).T            # (3N, nev), index 3 p + b
    assert np.abs(phi.conj().T @ phi - np.eye(nev)).max() <= 1e-10
    res = np.linalg.norm(h0 @ phi - phi * E[None, :], axis=0)
    assert res.max() <= 1.01 * max(tol, 1e-12) + 1e-12
    if precision == "fp64":
        # the same orbital subspace (levels are non-degenerate up to the gap at nev)
        assert E_ref[nev] - E_ref[nev - 1] > 1e-4
        P = phi @ phi.conj().T
        Pr = phi_ref[:, :nev] @ phi_ref[:, :nev].T
        assert np.abs(P - Pr).max() <= 1e-6


def test_spin_free_restart_and_field_rejected():
    import paper_2607_08447_amd as hkp
    w, g = _case("dqd_small")
    a = hkp.solve(_t(w.V), w.h, 8, strain=_t(w.strain), nb=16, tol=1e-9, spin_free=True)
    b = hkp.solve(_t(w.V), w.h, 8, strain=_t(w.strain), nb=16, tol=1e-9, spin_free=True,
                  X0=a.psi)
    assert a.status == 0 and b.status == 0
    assert np.abs(a.E.cpu().numpy() - b.E.cpu().numpy()).max() <= 1e-9
    assert b.stats["iters"] < a.stats["iters"]
    with pytest.raises(hkp.HkpError):
        hkp.solve(_t(w.V), w.h, 8, strain=_t(w.strain), B=(0.0, 0.0, 0.5), nb=16, spin_free=True)


@pytest.mark.parametrize("M", [1, 6, 21])
def test_soi_matrix_vs_oracle(M):
    """The spin-orbit matrix of the GPU's own orbitals against the oracle's formula on
    them, and the spectrum of diag(E) + SOI against the oracle's basis."""
    import paper_2607_08447_amd as hkp
    w, g = _case("fin_small")
    nev = 22
    r = hkp.solve(_t(w.V), w.h, nev, strain=_t(w.strain), nb=32, tol=1e-10, spin_free=True)
    assert r.status == 0
    phi = r.psi[:M]
    d = SI_MATERIAL["delta_so"]
    S = hkp.soi_matrix(phi, d).cpu().numpy()
    ph = phi.cpu().numpy().reshape(M, -1).T
    S_ref = soi_matrix(ph, d)
    assert np.abs(S - S_ref).max() <= 1e-12 * max(1.0, np.abs(S_ref).max())
    H = hkp.soi_matrix(phi, d, E=r.E[:M]).cpu().numpy()
    assert np.abs(H - single_particle(r.E[:M].cpu().numpy(), ph, d)).max() <= 1e-12
    # basis-invariant: the spectrum with the oracle's own orbitals
    h0 = h0_orbital(g, SI_MATERIAL, V=w.V, strain=w.strain)
    E_ref, phi_ref = lowest_arpack(h0, nev, tol=1e-14)
    if M < nev and E_ref[M] - E_ref[M - 1] > 1e-4:
        ev = np.linalg.eigvalsh(H)
        ev_ref = np.linalg.eigvalsh(single_particle(E_ref[:M], phi_ref[:, :M], d))
        assert np.abs(ev - ev_ref).max() <= 1e-8
    assert abs(np.trace(S).real - 2 * M * d / 3) <= 1e-12


def test_spin_free_full_size_properties():
    """256 x 48 x 48 double dot at B = 0 (strain on), 16 orbitals, FP64: sampled rows of
    the oracle's orbital block on the returned orbitals bounded by the residuals;
    the spin-orbit matrix Hermitian with trace 2 M Delta/3 and a Kramers-degenerate
    single-particle spectrum."""
    import paper_2607_08447_amd as hkp
    w, g = _case("dqd_256x48x48")
    print("spin-free dqd_256x48x48", flush=True)
    r = hkp.solve(_t(w.V), w.h, 16, strain=_t(w.strain), nb=24, tol=1e-8, spin_free=True)
    assert r.status == 0
    E = r.E.cpu().numpy()
    R = r.resid.cpu().numpy()
    assert R.max() <= 1e-8
    h0 = h0_orbital(g, SI_MATERIAL, V=w.V, strain=w.strain)
    rows = np.random.default_rng(3).choice(h0.shape[0], 4000, replace=False)
    Hr = h0[rows]
    for n in (0, 15):
        phi = r.psi[n].cpu().numpy().reshape(-1)
        res = Hr @ phi - E[n] * phi[rows]
        assert np.abs(res).max() <= R[n] * 1.01 + 1e-12
    d = SI_MATERIAL["delta_so"]
    H = hkp.soi_matrix(r.psi, d, E=r.E).cpu().numpy()
    assert np.abs(H - H.conj().T).max() <= 1e-13
    ev = np.linalg.eigvalsh(H)
    # time reversal maps the orbital subspace onto itself only up to the orbitals'
    # residuals (<= 1e-8 eV): pairs agree to that order
    assert np.abs(ev[0::2] - ev[1::2]).max() <= 1e-8
    assert abs(np.trace(H).real - (2 * E.sum() + 2 * 16 * d / 3)) <= 1e-9


@pytest.mark.parametrize("shape,precision", [("1,1,1", "fp64"), ("2,2,1", "fp64"),
                                             ("4,1,0", "fp64"), ("2,1,1,2", "fp64"),
                                             ("2,1,1", "mixed"), ("1,4,0", "mixed")])
def test_spin_free_stencil_launch_shapes(shape, precision, monkeypatch):
    """Every launch shape of the spin-free (three-component) stencil -- tile height,
    vector groups, row DMA, z split -- gives the oracle's orbital energies."""
    import paper_2607_08447_amd as hkp
    monkeypatch.setenv("HKP_STENCIL", shape)
    w, g = _case("dqd_small")
    tol, bar = (1e-9, 1e-8) if precision == "fp64" else (1e-6, 1e-6)
    r = hkp.solve(_t(w.V), w.h, 8, strain=_t(w.strain), nb=16, tol=tol, precision=precision,
                  spin_free=True, return_psi=False)
    assert r.status == 0
    E_ref, _ = lowest_arpack(h0_orbital(g, SI_MATERIAL, V=w.V, strain=w.strain), 8, tol=1e-14)
    assert np.abs(r.E.cpu().numpy() - E_ref).max() <= bar
