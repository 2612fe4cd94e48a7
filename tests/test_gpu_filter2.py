"""GPU parity of the two-step Chebyshev pass (temporal blocking of the FP32
filter), through the C ABI, against the oracle's assembled H (|J m_j> basis,
symmetric gauge):

    Y1 = a0 (H - c0) X + b0 Y_old,   Y2 = a1 (H - c1) Y1 + b1 X.

Coefficients as in the filter: a (H - c) maps the spectrum into [-1, 1], so the
FP32 rounding of Y1 is not amplified by the second step.  Tolerances: Y1 as
one FP32 step (3e-6 of max|Y|), Y2 twice that (its input carries Y1's
rounding).  Cases cover ragged y tiles, nz = 1, both field kinds the kernel
runs (B = 0; B with Bz = 0), strain on and off, every tile shape, and the
fallbacks to two one-step passes (Bz != 0; nx not a multiple of 16)."""

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid, hamiltonian_j, lowest_dense
from synth import random_block

pytestmark = pytest.mark.gpu

CASES = [
    # (name, shape, h, strain, B, passes)
    ("ragged_y_field_x", (32, 13, 7), 0.4, True, (0.5, 0.0, 0.0), 1),
    ("zero_field_no_strain", (16, 8, 5), 0.5, False, (0.0, 0.0, 0.0), 1),
    ("field_xy_strain", (48, 20, 9), 0.4, True, (0.6, -0.4, 0.0), 1),
    ("single_row", (16, 1, 4), 0.5, True, (0.0, 0.8, 0.0), 1),
    ("single_plane", (32, 9, 1), 0.5, True, (0.5, 0.0, 0.0), 1),
    ("fallback_bz", (32, 9, 6), 0.4, True, (0.3, 0.0, 0.7), 2),
    ("fallback_nx", (20, 9, 6), 0.4, True, (0.5, 0.0, 0.0), 2),
]

COEF = dict(alpha=(0.12, 0.11), shift=(8.4, 8.1), beta=(-0.9, -1.0))


def _fields(shape, strain, seed):
    r = np.random.default_rng(seed)
    V = 0.05 * r.standard_normal(shape)
    e = 2e-3 * r.standard_normal(shape + (6,)) if strain else None
    return V, e


def _run(shape, h, strain, B, seed, nvec=3, with_old=True):
    import torch
    import paper_2607_08447_amd as hkp
    V, e = _fields(shape, strain, seed)
    N = int(np.prod(shape))
    X = random_block(N * 6, nvec, seed=seed + 1)
    Yold = random_block(N * 6, nvec, seed=seed + 2) if with_old else None
    blk = lambda A: torch.from_numpy(A.reshape((nvec,) + shape + (6,)))
    beta = COEF["beta"] if with_old else (0.0, COEF["beta"][1])
    Y1, Y2, passes = hkp.filter_step2(torch.from_numpy(V), h, blk(X),
                                      None if Yold is None else blk(Yold),
                                      alpha=COEF["alpha"], shift=COEF["shift"], beta=beta,
                                      strain=None if e is None else torch.from_numpy(e), B=B)
    torch.cuda.synchronize()
    H = hamiltonian_j(Grid(*shape, h), SI_MATERIAL, V.ravel(),
                      None if e is None else e.reshape(-1, 6), B)
    a, c = COEF["alpha"], COEF["shift"]
    R1 = a[0] * (H @ X.T - c[0] * X.T)
    if with_old:
        R1 = R1 + beta[0] * Yold.T
    R2 = a[1] * (H @ R1 - c[1] * R1) + beta[1] * X.T
    err1 = np.abs(Y1.cpu().numpy().reshape(nvec, -1) - R1.T).max() / np.abs(R1).max()
    err2 = np.abs(Y2.cpu().numpy().reshape(nvec, -1) - R2.T).max() / np.abs(R2).max()
    return err1, err2, passes


@pytest.mark.parametrize("name,shape,h,strain,B,passes", CASES, ids=[c[0] for c in CASES])
def test_two_step_matches_oracle(name, shape, h, strain, B, passes):
    print(f"two-step case {name} {shape} B {B}", flush=True)
    err1, err2, p = _run(shape, h, strain, B, seed=40)
    assert p == passes, f"{name}: {p} passes, expected {passes}"
    assert err1 < 3e-6, f"{name}: Y1 rel err {err1:.3e}"
    assert err2 < 6e-6, f"{name}: Y2 rel err {err2:.3e}"


def test_two_step_without_old_block():
    """beta0 = 0 and no Y_old (the kernel must not read it)."""
    err1, err2, p = _run((32, 10, 6), 0.4, True, (0.5, 0.0, 0.0), seed=50, with_old=False)
    assert p == 1
    assert err1 < 3e-6 and err2 < 6e-6, (err1, err2)


TILES = [(16, 12), (16, 8), (32, 8)]


@pytest.mark.parametrize("tx,ty", TILES, ids=[f"{t[0]}x{t[1]}" for t in TILES])
def test_two_step_tiles(tx, ty, monkeypatch):
    """Every tile shape the autotuner may pick, on grids with ragged y tiles
    (ny not a multiple of the tile height), one vector per workgroup group."""
    monkeypatch.setenv("HKP_STENCIL2", f"{tx},{ty}")
    for k, (shape, strain, B) in enumerate([((64, 19, 7), True, (0.5, 0.0, 0.0)),
                                            ((32, 10, 5), False, (0.0, 0.0, 0.0))]):
        print(f"two-step tile {tx}x{ty} shape {shape}", flush=True)
        err1, err2, p = _run(shape, 0.4, strain, B, seed=60 + k, nvec=2)
        assert p == 1
        assert err1 < 3e-6 and err2 < 6e-6, (shape, err1, err2)


@pytest.mark.parametrize("tile", ["16,8", "16,12"])
def test_mixed_solve_with_two_step_passes(tile, monkeypatch):
    """A mixed-precision solve whose FP32 filter runs in two-step passes (forced
    tile; the passes carry the three-term recurrence, the default) gives the oracle's
    eigenvalues within 1 ueV (dense LAPACK on the assembled H), and the passes
    were used."""
    import torch
    import paper_2607_08447_amd as hkp
    monkeypatch.setenv("HKP_STENCIL2", tile)
    shape, h = (16, 7, 6), 0.5
    r = np.random.default_rng(70)
    x = (np.arange(shape[0]) - 7.5) * h
    y = (np.arange(shape[1]) - 3.0) * h
    z = (np.arange(shape[2]) - 2.5) * h
    X3, Y3, Z3 = np.meshgrid(x, y, z, indexing="ij")
    V = 0.02 * (X3 ** 2 + Y3 ** 2 + Z3 ** 2) + 0.002 * r.standard_normal(shape)
    e = np.zeros(shape + (6,))
    e[..., 2] = -3e-3
    B = (0.5, 0.0, 0.0)
    print(f"mixed solve with two-step tile {tile}", flush=True)
    res = hkp.solve(torch.from_numpy(V), h, 8, strain=torch.from_numpy(e), B=B, nb=16,
                    tol=1e-5, precision="mixed", return_psi=False)
    assert res.status == 0
    assert res.stats["n_stencil32x2"] > 0
    H = hamiltonian_j(Grid(*shape, h), SI_MATERIAL, V.ravel(), e.reshape(-1, 6), B)
    E_ref, _ = lowest_dense(H, 8)
    err = np.abs(res.E.cpu().numpy() - E_ref).max()
    assert err <= 1e-6, err
