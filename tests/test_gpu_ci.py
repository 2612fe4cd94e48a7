"""GPU parity of the two-hole configuration interaction (pair densities, their
grounded-electrode potentials from one batched Poisson solve, Coulomb
integrals, Slater-Condon matrix, spectrum, exchange J) against the CPU oracle,
through the C ABI.

Bars: with the GPU's own orbitals fed to both sides, Coulomb integrals within
1e-9 of their largest value, the determinant matrix within 1e-9 eV, the spectrum
and J within 1e-9 eV; against the oracle's own orbitals (the spectrum depends
only on the orbital space) within 1e-8 eV.  At full size: Hermiticity,
reciprocity and conjugation of the integrals, positive self-interaction,
orthonormal eigenvectors.
"""

import numpy as np
import pytest

from oracle import (SI_MATERIAL, Grid, ci_hamiltonian, coulomb_integrals, exchange, h0_orbital,
                    pair_densities, pair_potentials, poisson_solve, restrict, single_particle)
from oracle.solve import lowest_arpack
from synth import sp_device

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a))


def _setup(name):
    d = sp_device(name)
    phi0 = poisson_solve(d.pshape, d.h, d.eps_r, d.dirichlet, d.phi_fixed, np.zeros(d.pshape))
    V = d.V_off + restrict(phi0, d.shape, d.offset)
    return d, V


@pytest.mark.parametrize("name,M", [("sp_tiny", 1), ("sp_tiny", 2), ("sp_tiny", 4),
                                    ("sp_dqd_small", 5)])
def test_ci_vs_oracle(name, M):
    import paper_2607_08447_amd as hkp
    d, V = _setup(name)
    print(f"ci {name} M={M}", flush=True)
    r = hkp.solve(_t(V), d.h, M, strain=_t(d.strain), nb=M + 8, tol=1e-11, spin_free=True)
    assert r.status == 0
    ci = hkp.ci_solve(r.psi, r.E, d.h, d.pshape, d.offset, _t(d.eps_r), _t(d.dirichlet),
                      cg_tol=1e-13, return_vectors=True, return_matrix=True, return_coulomb=True)
    assert ci.status == 0 and ci.stats["determinants"] == M * (2 * M - 1)
    phi = r.psi.cpu().numpy().reshape(M, -1).T
    E = r.E.cpu().numpy()
    rho = pair_densities(phi, d.shape, d.h)
    Vp = pair_potentials(rho, d.pshape, d.offset, d.h, d.eps_r, d.dirichlet)
    C = coulomb_integrals(rho, Vp, d.shape, d.offset, d.h)
    Cg = ci.coulomb.cpu().numpy()
    print(f"max |C| {np.abs(C).max():.3e}, max |dC| {np.abs(Cg - C).max():.3e}", flush=True)
    assert np.abs(Cg - C).max() <= 1e-9 * np.abs(C).max()
    H = ci_hamiltonian(single_particle(E, phi, SI_MATERIAL["delta_so"]), C)
    assert np.abs(ci.H.cpu().numpy() - H).max() <= 1e-9
    ev = np.linalg.eigvalsh(H)
    assert np.abs(ci.E.cpu().numpy() - ev).max() <= 1e-9
    if M >= 2:
        assert abs(ci.J - exchange(ev)) <= 1e-9
    else:   # one orbital: a single determinant, no exchange splitting to report
        assert len(ev) == 1 and np.isnan(ci.J)
    U = ci.vectors.cpu().numpy()
    assert np.abs(U.conj().T @ U - np.eye(len(ev))).max() <= 1e-10
    assert np.abs(H @ U - U * ci.E.cpu().numpy()[None, :]).max() <= 1e-9
    # the oracle's own orbitals span the same space: the same spectrum
    Eo, phio = lowest_arpack(h0_orbital(Grid(*d.shape, d.h), SI_MATERIAL, V=V, strain=d.strain),
                             M + 1, tol=1e-14)
    if Eo[M] - Eo[M - 1] > 1e-4:
        rho_o = pair_densities(phio[:, :M], d.shape, d.h)
        C_o = coulomb_integrals(rho_o, pair_potentials(rho_o, d.pshape, d.offset, d.h, d.eps_r,
                                                       d.dirichlet), d.shape, d.offset, d.h)
        ev_o = np.linalg.eigvalsh(ci_hamiltonian(
            single_particle(Eo[:M], phio[:, :M], SI_MATERIAL["delta_so"]), C_o))
        assert np.abs(ci.E.cpu().numpy() - ev_o).max() <= 1e-8


def test_ci_full_size_properties():
    """The 256 x 48 x 48 double-dot fin in its 1.53M-node box (hole-free potential,
    B = 0, strain): 4 spin-free orbitals, 28 determinants."""
    import paper_2607_08447_amd as hkp
    d = sp_device("sp_dqd_256x48x48")
    print("ci sp_dqd_256x48x48 M=4", flush=True)
    # the hole-free potential from the GPU Poisson solve (a direct CPU solve of the
    # 1.53M-node box would take minutes)
    phi0, _, _, code = hkp.poisson(_t(d.eps_r), _t(d.dirichlet), _t(d.phi_fixed), None, d.h,
                                   tol=1e-12)
    assert code == 0
    ox, oy, oz = d.offset
    V = _t(d.V_off).cuda() + phi0[ox:ox + d.shape[0], oy:oy + d.shape[1], oz:oz + d.shape[2]]
    r = hkp.solve(V, d.h, 4, strain=_t(d.strain), nb=12, tol=1e-9, spin_free=True)
    assert r.status == 0
    ci = hkp.ci_solve(r.psi, r.E, d.h, d.pshape, d.offset, _t(d.eps_r), _t(d.dirichlet),
                      cg_tol=1e-11, return_vectors=True, return_matrix=True, return_coulomb=True)
    print({k: ci.stats[k] for k in ("cg_iters", "cg_relres", "t_poisson", "seconds")},
          f"J {ci.J:.4e} eV", flush=True)
    assert ci.status == 0 and ci.stats["determinants"] == 28
    C = ci.coulomb.cpu().numpy()
    scale = np.abs(C).max()
    assert np.abs(C - C.transpose(2, 3, 0, 1)).max() <= 1e-8 * scale
    assert np.abs(C - C.transpose(1, 0, 3, 2).conj()).max() <= 1e-8 * scale
    for i in range(4):
        assert C[i, i, i, i].real > 0
    H = ci.H.cpu().numpy()
    assert np.abs(H - H.conj().T).max() <= 1e-12
    U = ci.vectors.cpu().numpy()
    assert np.abs(U.conj().T @ U - np.eye(28)).max() <= 1e-10
    assert np.isfinite(ci.J)
