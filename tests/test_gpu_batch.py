"""Batched sweep (one launch per kernel over all Hamiltonians, optionally
recorded as a hipGraph) against the same Hamiltonians solved one by one, and
graph replay against eager execution."""

import numpy as np
import pytest

from synth import workload
from synth.inputs import coords, gaussian_gate

pytestmark = pytest.mark.gpu


def _sweep(nbatch=4):
    w = workload("dqd_small")
    x, _, _, c = coords(w.shape, w.h)
    bump = gaussian_gate(x, c[0])[:, None, None]
    Vs = np.stack([w.V + (0.01 * k) * bump for k in range(nbatch)])
    return w, Vs


@pytest.mark.parametrize("graph", [False, True])
def test_batch_fp64_equals_individual_solves(graph):
    import torch
    import paper_2607_08447_amd as hkp
    w, Vs = _sweep()
    nev = 8
    print(f"batch graph={graph}", flush=True)
    rb = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=torch.from_numpy(w.strain), B=w.B,
                         nb=16, tol=1e-9, graph=graph, return_psi=True)
    assert rb.status == 0
    Eb = rb.E.cpu().numpy()
    assert rb.resid.cpu().numpy().max() <= 1e-9
    for k in range(Vs.shape[0]):
        r1 = hkp.solve(torch.from_numpy(Vs[k]), w.h, nev, strain=torch.from_numpy(w.strain),
                       B=w.B, nb=16, tol=1e-9)
        assert np.abs(r1.E.cpu().numpy() - Eb[k]).max() <= 1e-8
    # the batched eigenvectors are eigenvectors of their own Hamiltonian
    psi = rb.psi
    for k in range(Vs.shape[0]):
        Hpsi = hkp.apply(torch.from_numpy(Vs[k]), w.h, psi[k], strain=torch.from_numpy(w.strain),
                         B=w.B)
        r = torch.linalg.vector_norm((Hpsi - rb.E[k][:, None, None, None, None] * psi[k])
                                     .reshape(nev, -1), dim=1)
        assert float(r.max()) <= 1e-8


def test_batch_mixed_graph_within_1ueV():
    import torch
    import paper_2607_08447_amd as hkp
    w, Vs = _sweep()
    nev = 8
    rb = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=torch.from_numpy(w.strain), B=w.B,
                         nb=16, tol=1e-6, graph=True, precision="mixed")
    assert rb.status == 0
    ref = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=torch.from_numpy(w.strain),
                          B=w.B, nb=16, tol=1e-10, graph=False)
    assert np.abs(rb.E.cpu().numpy() - ref.E.cpu().numpy()).max() <= 1e-6
    assert rb.stats["n_hx_fp32"] > 0


def test_graph_single_equals_eager():
    import torch
    import paper_2607_08447_amd as hkp
    w = workload("fin_small")
    a = hkp.solve(torch.from_numpy(w.V), w.h, 8, strain=torch.from_numpy(w.strain), B=w.B, nb=16,
                  tol=1e-9, graph=False)
    b = hkp.solve(torch.from_numpy(w.V), w.h, 8, strain=torch.from_numpy(w.strain), B=w.B, nb=16,
                  tol=1e-9, graph=True)
    assert a.status == 0 and b.status == 0
    assert np.abs(a.E.cpu().numpy() - b.E.cpu().numpy()).max() <= 1e-9


def test_batch_warm_start_equals_cold():
    """A batch restarted from its own eigenvectors (HKP_FLAG_X0_NEV: nev given
    vectors, the rest of each block random) and from whole given blocks
    reaches the cold-start eigenvalues, the warm restart in fewer iterations."""
    import torch
    import paper_2607_08447_amd as hkp
    w, Vs = _sweep(3)
    nev, nb = 8, 16
    S = torch.from_numpy(w.strain)
    print("batch warm start (nev and nb initial vectors)", flush=True)
    cold = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=S, B=w.B, nb=nb, tol=1e-9,
                           graph=False, return_psi=True, psi_block=True)
    assert cold.status == 0
    assert tuple(cold.psi.shape) == (Vs.shape[0], nb) + w.shape + (6,)
    # the whole final block is orthonormal
    for k in range(Vs.shape[0]):
        Q = cold.psi[k].reshape(nb, -1)
        G = Q.conj() @ Q.T
        assert float((G - torch.eye(nb, dtype=G.dtype, device=G.device)).abs().max()) <= 1e-10
    warm = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=S, B=w.B, nb=nb, tol=1e-9,
                           graph=False, X0=cold.psi[:, :nev])
    assert warm.status == 0
    assert np.abs(warm.E.cpu().numpy() - cold.E.cpu().numpy()).max() <= 1e-8
    assert warm.resid.cpu().numpy().max() <= 1e-9
    assert warm.stats["iters"] < cold.stats["iters"]
    # restarted from its own converged blocks a batch is done after the first
    # Rayleigh-Ritz step
    again = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=S, B=w.B, nb=nb, tol=1e-9,
                            graph=False, X0=cold.psi)
    assert again.status == 0 and again.stats["iters"] == 0
    assert np.abs(again.E.cpu().numpy() - cold.E.cpu().numpy()).max() <= 1e-10
    g = torch.Generator(device="cuda").manual_seed(5)
    blk = torch.randn((Vs.shape[0], nb) + w.shape + (6,), dtype=torch.complex128, device="cuda",
                      generator=g)
    full = hkp.solve_batch(torch.from_numpy(Vs), w.h, nev, strain=S, B=w.B, nb=nb, tol=1e-9,
                           graph=True, X0=blk)
    assert full.status == 0
    assert np.abs(full.E.cpu().numpy() - cold.E.cpu().numpy()).max() <= 1e-8


def test_single_warm_start_from_neighbour():
    """One solve started from the eigenvectors of a neighbouring potential (as
    between Schroedinger-Poisson iterations) equals the cold solve."""
    import torch
    import paper_2607_08447_amd as hkp
    w, Vs = _sweep(2)
    S = torch.from_numpy(w.strain)
    r0 = hkp.solve(torch.from_numpy(Vs[0]), w.h, 8, strain=S, B=w.B, nb=16, tol=1e-9,
                   psi_block=True)
    assert tuple(r0.psi.shape) == (16,) + w.shape + (6,)
    cold = hkp.solve(torch.from_numpy(Vs[1]), w.h, 8, strain=S, B=w.B, nb=16, tol=1e-9)
    assert r0.status == 0 and cold.status == 0
    for X0 in (r0.psi[:8], r0.psi):      # nev vectors + random, the whole block
        warm = hkp.solve(torch.from_numpy(Vs[1]), w.h, 8, strain=S, B=w.B, nb=16, tol=1e-9,
                         X0=X0)
        assert warm.status == 0
        assert np.abs(warm.E.cpu().numpy() - cold.E.cpu().numpy()).max() <= 1e-8
        assert warm.resid.cpu().numpy().max() <= 1e-9
        assert warm.stats["iters"] < cold.stats["iters"]


@pytest.mark.parametrize("precision,tol,bar", [("fp64", 1e-9, 1e-8), ("mixed", 1e-6, 1e-6)])
def test_sweep_continuation_equals_batch(precision, tol, bar):
    """solve_sweep (every 3rd member cold, the others warm-started from the
    nearest of them) against the cold batched solve of the same sweep."""
    import torch
    import paper_2607_08447_amd as hkp
    w, Vs = _sweep(7)
    S = torch.from_numpy(w.strain)
    print(f"sweep continuation {precision}", flush=True)
    ref = hkp.solve_batch(torch.from_numpy(Vs), w.h, 8, strain=S, B=w.B, nb=16, tol=1e-10,
                          graph=False)
    sw = hkp.solve_sweep(torch.from_numpy(Vs), w.h, 8, strain=S, B=w.B, nb=16, tol=tol,
                         precision=precision, stride=3, return_psi=True)
    assert sw.status == 0
    assert set(sw.stats) == {"anchors", "rest"}
    assert np.abs(sw.E.cpu().numpy() - ref.E.cpu().numpy()).max() <= bar
    assert sw.resid.cpu().numpy().max() <= tol
    # member k's returned vectors are its own eigenvectors
    for k in (1, 5):
        Hpsi = hkp.apply(torch.from_numpy(Vs[k]), w.h, sw.psi[k], strain=S, B=w.B)
        r = torch.linalg.vector_norm((Hpsi - sw.E[k][:, None, None, None, None] * sw.psi[k])
                                     .reshape(8, -1), dim=1)
        assert float(r.max()) <= tol * 1.01
