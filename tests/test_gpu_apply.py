"""GPU parity of the matrix-free Hamiltonian application and the fused
Chebyshev step, through the C ABI, against the oracle's assembled H (|J m_j>
basis, symmetric gauge).

Tolerances: FP64 -- every output is a sum of ~40 products bounded by |H| |x|,
so the rounding error is a few 1e-15 of max|Y|; 1e-13 leaves margin for the
gauge/basis transforms.  FP32 stencil -- operands and arithmetic rounded to
FP32 (2^-24 = 6e-8 relative), the same ~40-term sums: 3e-6 of max|Y|.
"""

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid, hamiltonian_j
from synth import random_block, workload

pytestmark = pytest.mark.gpu

CASES = [
    # (name, shape, h, strain, B)
    ("harmonic", (10, 8, 8), 0.5, False, (0.0, 0.0, 0.0)),
    ("ragged_general_B", (17, 9, 5), 0.4, True, (0.7, -1.1, 0.9)),
    ("three_x_tiles", (130, 5, 3), 0.4, True, (0.5, 0.0, 0.0)),
    ("several_tiles", (70, 12, 10), 0.4, True, (0.5, 0.0, 0.0)),
    ("exact_tile", (64, 4, 4), 0.5, False, (0.0, 0.3, 0.0)),
    ("chain_nx1", (1, 1, 7), 0.5, True, (0.0, 0.0, 0.2)),
    ("plane_nz1", (9, 6, 1), 0.5, True, (0.0, 0.0, 0.0)),
]


def _fields(shape, h, strain, seed):
    r = np.random.default_rng(seed)
    V = 0.05 * r.standard_normal(shape)
    e = 2e-3 * r.standard_normal(shape + (6,)) if strain else None
    return V, e


def _oracle_H(shape, h, V, e, B):
    g = Grid(*shape, h)
    return hamiltonian_j(g, SI_MATERIAL, V.ravel(), None if e is None else e.reshape(-1, 6), B)


@pytest.mark.parametrize("name,shape,h,strain,B", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("mixed", 3e-6)])
def test_apply_matches_oracle(name, shape, h, strain, B, precision, tol):
    import torch
    import paper_2607_08447_amd as hkp
    V, e = _fields(shape, h, strain, 1)
    nvec = 3
    N = int(np.prod(shape))
    X = random_block(N * 6, nvec, seed=2)
    print(f"case {name} {shape} {precision}", flush=True)
    Y = hkp.apply(torch.from_numpy(V), h, torch.from_numpy(X.reshape((nvec,) + shape + (6,))),
                  strain=None if e is None else torch.from_numpy(e), B=B, precision=precision)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().reshape(nvec, -1)
    H = _oracle_H(shape, h, V, e, B)
    Yo = (H @ X.T).T
    err = np.abs(Yg - Yo).max() / np.abs(Yo).max()
    assert err < tol, f"{name} {precision}: rel err {err:.3e}"


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("mixed", 3e-6)])
def test_filter_step_matches_oracle(precision, tol):
    import torch
    import paper_2607_08447_amd as hkp
    shape, h, B = (33, 10, 7), 0.4, (0.5, 0.2, -0.3)
    V, e = _fields(shape, h, True, 3)
    N = int(np.prod(shape))
    nvec = 2
    X = random_block(N * 6, nvec, seed=4)
    Yold = random_block(N * 6, nvec, seed=5)
    alpha, shift, beta = 0.37, 4.2, -0.81
    Y = hkp.filter_step(torch.from_numpy(V), h, torch.from_numpy(X.reshape((nvec,) + shape + (6,))),
                        torch.from_numpy(Yold.reshape((nvec,) + shape + (6,))), alpha, shift, beta,
                        strain=torch.from_numpy(e), B=B, precision=precision)
    Yg = Y.cpu().numpy().reshape(nvec, -1)
    H = _oracle_H(shape, h, V, e, B)
    Yo = (alpha * (H @ X.T - shift * X.T) + beta * Yold.T).T
    err = np.abs(Yg - Yo).max() / np.abs(Yo).max()
    assert err < tol, f"rel err {err:.3e}"


def test_apply_full_size_sampled_rows():
    """The fin workload at its full size (128 x 40 x 40, strain, B = 0.5 T):
    sampled rows of H X computed one by one by the oracle."""
    import torch
    import paper_2607_08447_amd as hkp
    w = workload("fin_qd_128x40x40")
    N = w.npts
    X = random_block(N * 6, 1, seed=6)
    Y = hkp.apply(torch.from_numpy(w.V), w.h, torch.from_numpy(X.reshape((1,) + w.shape + (6,))),
                  strain=torch.from_numpy(w.strain), B=w.B)
    Yg = Y.cpu().numpy().reshape(-1)
    H = _oracle_H(w.shape, w.h, w.V, w.strain, w.B)
    rows = np.random.default_rng(7).choice(N * 6, 4000, replace=False)
    Yo = H[rows] @ X[0]
    err = np.abs(Yg[rows] - Yo).max() / np.abs(Yo).max()
    assert err < 1e-13


VARIANTS = [(ty, vg, dma, zs) for zs in (0, 2) for dma in (0, 1) for vg in (1, 2, 4)
            for ty in (1, 2, 4)]
VARIANT_SHAPES = [
    # x spans whole 64-wide tiles (the row-DMA variant applies); y ragged for every tile
    # height; nz >= 8 on two grids so that a forced z split takes effect (odd and even nz)
    ((128, 7, 5), 0.4, True, (0.5, 0.0, 0.0)),
    ((64, 9, 11), 0.5, True, (0.7, -1.1, 0.9)),
    ((192, 3, 8), 0.4, False, (0.0, 0.0, 0.0)),
]


@pytest.mark.parametrize("ty,vg,dma,zs", VARIANTS,
                         ids=[f"ty{v[0]}_g{v[1]}_dma{v[2]}_z{v[3]}" for v in VARIANTS])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("mixed", 3e-6)])
def test_stencil_launch_variants(ty, vg, dma, zs, precision, tol, monkeypatch):
    """Every launch shape the stencil may run with (tile height, vectors per
    tile group -- 3 vectors, so groups of 2 leave a ragged last group and 4
    clamps to tile-major --, global->LDS row staging, and the split of each
    column march into two z ranges) gives the oracle's
    alpha (H - shift) X + beta Y_old."""
    import torch
    import paper_2607_08447_amd as hkp
    monkeypatch.setenv("HKP_STENCIL", f"{ty},{vg},{dma},{zs}")
    for k, (shape, h, strain, B) in enumerate(VARIANT_SHAPES):
        V, e = _fields(shape, h, strain, 10 + k)
        N = int(np.prod(shape))
        nvec = 3
        X = random_block(N * 6, nvec, seed=20 + k)
        Yold = random_block(N * 6, nvec, seed=30 + k)
        alpha, shift, beta = 0.6, 1.3, -0.5
        print(f"variant ty {ty} vgroup {vg} dma {dma} zsplit {zs} {precision} shape {shape}",
              flush=True)
        Y = hkp.filter_step(torch.from_numpy(V), h,
                            torch.from_numpy(X.reshape((nvec,) + shape + (6,))),
                            torch.from_numpy(Yold.reshape((nvec,) + shape + (6,))), alpha, shift,
                            beta, strain=None if e is None else torch.from_numpy(e), B=B,
                            precision=precision)
        Yg = Y.cpu().numpy().reshape(nvec, -1)
        H = _oracle_H(shape, h, V, e, B)
        Yo = (alpha * (H @ X.T - shift * X.T) + beta * Yold.T).T
        err = np.abs(Yg - Yo).max() / np.abs(Yo).max()
        assert err < tol, f"{shape} {precision}: rel err {err:.3e}"
