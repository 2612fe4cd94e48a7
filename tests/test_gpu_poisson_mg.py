"""The Poisson CG's multigrid preconditioner, pinned iterate by iterate.

The converged potential is pinned elsewhere (the oracle's direct solve); a wrong
but still positive-definite preconditioner would pass that check and only cost
iterations.  Here a plain numpy restatement of the library's V-cycle -- 2 x 2 x 2
aggregation with Galerkin coarse operators, damped Jacobi (w = 0.9) before and
after each coarse correction, the finest correction scaled by 1.8, 30 Jacobi
sweeps from zero on the coarsest level (the first level past the finest with at
most 256 nodes) -- runs inside textbook preconditioned CG from the same start,
and the GPU's potential after the same small number of iterations must agree to
rounding.  The boxes cover the per-level kernels, the one-workgroup tail with
one, two and three levels, ragged (odd) aggregates, and the CG update fused into
the finest restriction.  The operator comes from the oracle's Poisson matrix.
"""

import numpy as np
import pytest

from oracle import E_OVER_EPS0, poisson_operator

W, ALPHA0, SWEEPS, COARSEST = 0.9, 1.8, 30, 256


def _box(shape, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, 12.0, shape)
    rho = rng.normal(0.0, 1e-2, shape)
    dirichlet = np.zeros(shape, dtype=np.uint8)
    dirichlet[..., -1][rng.uniform(size=shape[:2]) < 0.3] = 1
    dirichlet[0, 0, 0] = 1
    phi_fixed = np.where(dirichlet == 1, rng.uniform(-0.3, 0.3, shape), 0.0)
    return eps, dirichlet, phi_fixed, rho


def _links(shape, h, eps, free):
    """Free-free link weights along +x, +y, +z per node (0 past the box or towards
    an electrode) and the diagonal (every in-box link of a free node) from the
    oracle's operator."""
    L = poisson_operator(shape, h, eps).tocsr()
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    a = []
    for axis in range(3):
        w = np.zeros(shape)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, shape[axis] - 1)
        hi[axis] = slice(1, shape[axis])
        i, j = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        c = -np.asarray(L[i, j]).ravel()
        c = np.where(free.ravel()[i] & free.ravel()[j], c, 0.0)
        w[tuple(lo)] = c.reshape(w[tuple(lo)].shape)
        a.append(w)
    diag = np.where(free, L.diagonal().reshape(shape), 0.0)
    return a, diag


def _apply(a, diag, u):
    out = diag * u
    for axis in range(3):
        n = u.shape[axis]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        out[lo] -= a[axis][lo] * u[hi]
        out[hi] -= a[axis][lo] * u[lo]
    return out


def _pad_even(v):
    return np.pad(v, [(0, s % 2) for s in v.shape])


def _aggregate(v):
    """Sum over the 2 x 2 x 2 children of every coarse node."""
    p = _pad_even(v)
    s = p.shape
    return p.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2).sum(axis=(1, 3, 5))


def _coarsen(a, diag):
    """Galerkin operator of the aggregation: links crossing an aggregate face add up,
    links inside an aggregate leave the diagonal (twice their weight)."""
    d = _aggregate(diag)
    ca = []
    for axis in range(3):
        p = _pad_even(a[axis])
        sel = [slice(None)] * 3
        sel[axis] = slice(0, None, 2)
        inner = np.zeros_like(p)
        inner[tuple(sel)] = p[tuple(sel)]
        d = d - 2.0 * _aggregate(inner[tuple(slice(0, n) for n in a[axis].shape)])
        sel[axis] = slice(1, None, 2)
        outer = np.zeros_like(p)
        outer[tuple(sel)] = p[tuple(sel)]
        ca.append(_aggregate(outer[tuple(slice(0, n) for n in a[axis].shape)]))
    return ca, d


def _levels(a, diag):
    lv = [(a, diag)]
    while True:
        ca, cd = _coarsen(*lv[-1])
        lv.append((ca, cd))
        if cd.size <= COARSEST or cd.shape == (1, 1, 1):
            return lv


def _vcycle(lv, k, b):
    a, diag = lv[k]
    dinv = np.where(diag > 0.0, 1.0 / np.where(diag > 0.0, diag, 1.0), 0.0)
    active = dinv != 0.0
    if k == len(lv) - 1:
        u = np.zeros_like(b)
        for _ in range(SWEEPS):
            u = u + W * dinv * (b - _apply(a, diag, u))
        return u
    u_pre = W * dinv * b
    res = np.where(active, b - _apply(a, diag, u_pre), 0.0)
    e = _vcycle(lv, k + 1, _aggregate(res))
    pe = np.repeat(np.repeat(np.repeat(e, 2, 0), 2, 1), 2, 2)[tuple(slice(0, n) for n in b.shape)]
    up = np.where(active, u_pre + (ALPHA0 if k == 0 else 1.0) * pe, 0.0)
    return np.where(active, up + W * dinv * (b - _apply(a, diag, up)), 0.0)


def _pcg(shape, h, eps, dirichlet, phi_fixed, rho, iters):
    free = dirichlet == 0
    L = poisson_operator(shape, h, eps).tocsr()
    phi = np.where(free, 0.0, phi_fixed).ravel()   # zero start, electrodes imposed
    f = free.ravel()
    r = np.where(f, E_OVER_EPS0 * rho.ravel() - L @ phi, 0.0)   # = b at the zero start
    bb = float(r @ r)
    a, diag = _links(shape, h, eps, free)
    lv = _levels(a, diag)
    M = lambda v: _vcycle(lv, 0, v.reshape(shape)).ravel()
    z = M(r)
    rz = float(r @ z)
    p = np.zeros_like(r)
    beta = 0.0
    for _ in range(iters):
        p = z + beta * p
        q = np.where(f, L @ p, 0.0)
        alpha = rz / float(p @ q)
        phi = phi + alpha * p
        r = r - alpha * q
        z = M(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
    return phi.reshape(shape), np.sqrt(float(r @ r) / bb), len(lv)


CASES = [
    ("ragged_levels_and_tail", (37, 29, 23)),    # per-level kernels, a two-level tail
    ("thin_three_level_tail", (1, 1, 2000)),
    ("coarsest_only_tail", (40, 3, 2)),
    ("column", (1, 1, 9)),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,shape", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("iters", [1, 4])
def test_multigrid_pcg_iterates_match_restatement(name, shape, iters):
    import paper_2607_08447_amd as hkp
    import torch
    eps, dirichlet, phi_fixed, rho = _box(shape, 7 + sum(shape))
    prev = hkp.poisson_preconditioner("multigrid")
    try:
        print(f"multigrid pcg {name} {shape} iterations {iters}", flush=True)
        t = lambda v: torch.from_numpy(np.ascontiguousarray(v))
        phi, it, rel, _ = hkp.poisson(t(eps), t(dirichlet), t(phi_fixed), t(rho), 0.4,
                                      tol=1e-30, max_iter=iters)
    finally:
        hkp.poisson_preconditioner(prev)
    ref, rel_ref, nlev = _pcg(shape, 0.4, eps, dirichlet, phi_fixed, rho, iters)
    assert nlev >= 2 and it == iters
    err = np.abs(phi.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-9, (name, iters, err)
    assert abs(rel - rel_ref) <= 1e-8 * rel_ref, (rel, rel_ref)


def test_restatement_converges_to_the_oracle_solution():
    """The numpy restatement is itself a working preconditioner: its CG reaches the
    oracle's direct solution (so the comparison above is against a correct
    iteration, not a shared mistake)."""
    from oracle import poisson_solve
    shape = (17, 13, 11)
    eps, dirichlet, phi_fixed, rho = _box(shape, 3)
    ref = poisson_solve(shape, 0.4, eps, dirichlet, phi_fixed, rho)
    phi, rel, _ = _pcg(shape, 0.4, eps, dirichlet, phi_fixed, rho, 40)
    assert rel < 1e-12
    assert np.abs(phi - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.gpu
@pytest.mark.parametrize("precond", ["multigrid", "jacobi"])
def test_recorded_chunk_reused_with_new_coefficients_and_charge(precond):
    """hkp_poisson keeps its recorded CG chunk across calls that pass the same
    buffers.  The chunk must hold no coefficient or charge value: a second call on
    the same workspace, solution and mask buffers with another permittivity,
    charge and electrode potential, and a third with the first inputs again, each
    reach the oracle's direct solution (the electrode mask's contents change too;
    the mask buffer does not)."""
    import ctypes as C
    import torch
    import paper_2607_08447_amd as hkp
    from paper_2607_08447_amd import _lib as L
    from paper_2607_08447_amd.api import _pgrid, _private_stream
    from oracle import poisson_solve
    shape, h = (21, 14, 9), 0.4
    boxes = [_box(shape, 11), _box(shape, 12)]   # different electrodes too
    pg = _pgrid(shape)
    need = L.lib.hkp_poisson_workspace_bytes(C.byref(pg))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    dirm = torch.empty(shape, dtype=torch.uint8, device="cuda")
    eps_d = torch.empty(shape, dtype=torch.float64, device="cuda")
    rho_d = torch.empty(shape, dtype=torch.float64, device="cuda")
    fix_d = torch.empty(shape, dtype=torch.float64, device="cuda")
    phi = torch.empty(shape, dtype=torch.float64, device="cuda")
    s = _private_stream()
    prev = hkp.poisson_preconditioner(precond)
    try:
        for k in (0, 1, 0):
            eps, dirichlet, phi_fixed, rho = boxes[k]
            print(f"reused chunk {precond} call with box {k}", flush=True)
            dirm.copy_(torch.from_numpy(dirichlet))
            eps_d.copy_(torch.from_numpy(eps))
            rho_d.copy_(torch.from_numpy(rho))
            fix_d.copy_(torch.from_numpy(phi_fixed))
            phi.zero_()
            torch.cuda.synchronize()
            it = C.c_int32(0)
            rel = C.c_double(0.0)
            with torch.cuda.stream(s):
                code = L.lib.hkp_poisson(C.byref(pg), h, C.c_void_p(eps_d.data_ptr()),
                                         C.c_void_p(dirm.data_ptr()), C.c_void_p(fix_d.data_ptr()),
                                         C.c_void_p(rho_d.data_ptr()), C.c_void_p(phi.data_ptr()),
                                         1e-13, 20000, C.c_void_p(ws.data_ptr()), C.c_size_t(need),
                                         C.c_void_p(s.cuda_stream), C.byref(it), C.byref(rel))
            s.synchronize()
            assert code == 0 and rel.value <= 1e-13, (code, rel.value)
            ref = poisson_solve(shape, h, eps, dirichlet, phi_fixed, rho)
            err = np.abs(phi.cpu().numpy() - ref).max()
            assert err <= 1e-9 * max(1.0, np.abs(ref).max()), (k, err)
    finally:
        hkp.poisson_preconditioner(prev)
