"""Python binding of the hole k.p eigensolver (PyTorch supplies device memory
and streams; every step of the computation runs in the HIP library).

Layouts follow include/hkp.h: fields are float64 [nx, ny, nz] (strain with a
trailing Voigt axis of 6), spinor blocks complex128 [nvec, nx, ny, nz, 6] in
the |J m_j> basis and the symmetric gauge.
"""

import contextlib
import ctypes as C
import os
from dataclasses import dataclass

import torch

from . import _lib as L

SI = dict(gamma1=4.285, gamma2=0.339, gamma3=1.446, delta_so_eV=0.044, kappa=-0.42,
          a_v_eV=2.46, b_eV=-2.35, d_eV=-5.32)


def _material(m=None):
    mat = L.hkp_material()
    L.lib.hkp_default_material(C.byref(mat))
    if m:
        for k, v in m.items():
            k2 = {"delta_so": "delta_so_eV", "a_v": "a_v_eV", "b": "b_eV", "d": "d_eV"}.get(k, k)
            setattr(mat, k2, float(v))
    return mat


def _grid(shape, h):
    nx, ny, nz = (int(s) for s in shape)
    return L.hkp_grid(nx, ny, nz, float(h))


def _dev(x, dtype):
    """Device tensor (contiguous) of the given dtype; numpy arrays are copied over."""
    if x is None:
        return None
    if not torch.is_tensor(x):
        x = torch.as_tensor(x)
    if not x.is_cuda:
        x = x.to("cuda")
    return x.to(dtype).contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


_PRIVATE_STREAMS = {}


def _private_stream():
    """The library's own stream on the current device (default priority), made once:
    a stream's first use costs milliseconds, so calls do not take a new one each
    time.  Capturing a stream needs one that is not the legacy default stream."""
    dev = torch.cuda.current_device()
    s = _PRIVATE_STREAMS.get(dev)
    if s is None:
        s = _PRIVATE_STREAMS[dev] = torch.cuda.Stream(device=dev)
    return s


@contextlib.contextmanager
def _iter_callback(callback):
    """While the block runs, the eigensolves of this thread report to callback
    (None: nothing) after every outer iteration (every replayed chunk in graph
    mode): a dict with iter, batch, nb, nev and numpy arrays nconv [batch],
    fp64 [batch], ritz_eV and resid_eV [batch, nb].  A true return value ends the
    solve (status 1 unless every state converged); an exception raised by the
    callback ends it too and is raised again after the call."""
    if callback is None:
        yield
        return
    import numpy as np
    raised = []

    def _fn(pinfo, _user):
        try:
            i = pinfo.contents
            arr = lambda ptr, shape: np.ctypeslib.as_array(ptr, shape).copy()
            d = {"iter": i.iter, "batch": i.batch, "nb": i.nb, "nev": i.nev,
                 "nconv": arr(i.nconv, (i.batch,)), "fp64": arr(i.fp64, (i.batch,)),
                 "ritz_eV": arr(i.ritz_eV, (i.batch, i.nb)),
                 "resid_eV": arr(i.resid_eV, (i.batch, i.nb))}
            return 1 if callback(d) else 0
        except BaseException as e:   # noqa: BLE001 -- kept and raised after the solve
            raised.append(e)
            return 1

    fn = L.HKP_ITER_FN(_fn)
    L.lib.hkp_set_iter_callback(fn, None)
    try:
        yield
    finally:
        L.lib.hkp_set_iter_callback(L.HKP_ITER_FN(), None)
    if raised:
        raise raised[0]


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _B(B):
    return (C.c_double * 3)(*[float(b) for b in B])


@dataclass
class SolveResult:
    E: torch.Tensor          # [nev] or [batch, nev], eV
    psi: torch.Tensor        # [nev, nx, ny, nz, 6] complex128 (or batched), or None
    resid: torch.Tensor      # same leading shape as E, eV
    stats: dict
    status: int


def _opts(nev, nb, degree, max_iter, tol, precision, flags, seed):
    o = L.hkp_opts()
    L.lib.hkp_default_opts(C.byref(o))
    o.nev = int(nev)
    o.nb = int(nb)
    o.degree = int(degree)
    o.max_iter = int(max_iter)
    o.tol_eV = float(tol)
    o.precision = L.HKP_PREC_MIXED if precision in ("mixed", 1) else L.HKP_PREC_FP64
    o.flags = int(flags)
    o.seed = int(seed)
    return o


def workspace_bytes(shape, h, nev, nb=0, degree=0, precision="fp64", batch=1):
    g = _grid(shape, h)
    o = _opts(nev, nb, degree, 10, 1e-8, precision, 0, 1)
    n = L.lib.hkp_workspace_bytes(C.byref(g), C.byref(o), int(batch))
    if n == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    return int(n)


def _x0(X0, lead, nev, nb, shape, ncomp=6):
    """Initial-block flags and block size for X0 of shape lead + [k, nx, ny, nz, ncomp]:
    k = nev is a previous solve's psi (the rest of the block drawn at random),
    any other k is the whole block (nb = k)."""
    X0d = _dev(X0, torch.complex128)
    if X0d is None:
        return None, 0, nb
    if X0d.dim() != len(lead) + 5 or tuple(X0d.shape[:len(lead)]) != lead \
            or tuple(X0d.shape[len(lead) + 1:]) != shape + (ncomp,):
        raise ValueError(f"X0 must be {list(lead)} + [nev or nb, nx, ny, nz, {ncomp}]")
    k = X0d.shape[len(lead)]
    if k == nev:
        return X0d, L.HKP_FLAG_X0 | L.HKP_FLAG_X0_NEV, nb
    if nb and k != nb:
        raise ValueError(f"X0 holds {k} vectors: nev ({nev}) or nb ({nb}) expected")
    return X0d, L.HKP_FLAG_X0, k


def _npsi(g, o, nev, block):
    """Vectors written to psi: nev, or with block the whole block (flag set on o)."""
    if not block:
        return nev
    o.flags |= L.HKP_FLAG_PSI_BLOCK
    return int(L.lib.hkp_block_size(C.byref(g), C.byref(o)))


def solve(V, h, nev, strain=None, B=(0.0, 0.0, 0.0), nb=0, degree=0, tol=1e-8,
          precision="fp64", max_iter=200, seed=1, X0=None, graph=False, material=None,
          return_psi=True, workspace=None, polish=True, lock=True, psi_block=False,
          spin_free=False, cheb_product=False, callback=None):
    """Lowest `nev` eigenpairs of H for the potential V (float64 [nx, ny, nz], eV).

    spin_free=True solves the orbital problem H_0 without spin-orbit coupling
    (B must be zero): each orbital level once, psi (and X0) [n, nx, ny, nz, 3]
    holding the X, Y, Z components.

    X0 (optional, complex128): the whole initial block [nb, nx, ny, nz, 6], or
    [nev, nx, ny, nz, 6] -- a previous solve's psi -- completed with random
    vectors.  psi_block=True returns all nb final Ritz vectors as psi (the
    initial block of a later restart).  lock=False filters every vector of the
    block in every iteration (no soft locking of converged Kramers pairs).
    cheb_product=True evaluates the Chebyshev filter in product form over its
    roots instead of the three-term recurrence (the same polynomial; two blocks
    moved per step instead of three).  callback(progress) is called after every
    outer iteration (see _iter_callback); returning True ends the solve."""
    V = _dev(V, torch.float64)
    shape = tuple(V.shape)
    if len(shape) != 3:
        raise ValueError("V must be [nx, ny, nz]")
    strain = _dev(strain, torch.float64)
    g = _grid(shape, h)
    ncomp = 3 if spin_free else 6
    X0d, xflags, nb = _x0(X0, (), nev, nb, shape, ncomp)
    flags = (L.HKP_FLAG_GRAPH if graph else 0) | xflags | (L.HKP_FLAG_SPIN_FREE if spin_free else 0)
    if not polish:
        flags |= L.HKP_FLAG_NO_FP64_POLISH
    if not lock:
        flags |= L.HKP_FLAG_NO_LOCK
    if cheb_product:
        flags |= L.HKP_FLAG_CHEB_PRODUCT
    o = _opts(nev, nb, degree, max_iter, tol, precision, flags, seed)
    need = L.lib.hkp_workspace_bytes(C.byref(g), C.byref(o), 1)
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    npsi = _npsi(g, o, nev, return_psi and psi_block)
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    E = torch.empty(nev, dtype=torch.float64, device="cuda")
    R = torch.empty(nev, dtype=torch.float64, device="cuda")
    psi = torch.empty((npsi,) + shape + (ncomp,), dtype=torch.complex128, device="cuda") \
        if return_psi else None
    st = L.hkp_stats()
    stream_ctx = _private_stream() if graph else None
    mat = _material(material)
    if stream_ctx is not None:
        stream_ctx.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream_ctx), _iter_callback(callback):
            code = L.lib.hkp_solve(C.byref(g), C.byref(mat), C.byref(o), _ptr(V), _ptr(strain),
                                   _B(B), _ptr(X0d), _ptr(E), _ptr(psi), _ptr(R), _ptr(ws),
                                   C.c_size_t(ws.numel()), _stream(stream_ctx), C.byref(st))
        torch.cuda.current_stream().wait_stream(stream_ctx)
    else:
        with _iter_callback(callback):
            code = L.lib.hkp_solve(C.byref(g), C.byref(mat), C.byref(o), _ptr(V), _ptr(strain),
                                   _B(B), _ptr(X0d), _ptr(E), _ptr(psi), _ptr(R), _ptr(ws),
                                   C.c_size_t(ws.numel()), _stream(), C.byref(st))
    L.check(code)
    return SolveResult(E, psi, R, st.as_dict(), code)


def solve_batch(V, h, nev, strain=None, B=(0.0, 0.0, 0.0), nb=0, degree=0, tol=1e-8,
                precision="fp64", max_iter=200, seed=1, graph=True, material=None,
                return_psi=False, workspace=None, polish=True, lock=True, X0=None,
                psi_block=False, spin_free=False, cheb_product=False, callback=None):
    """Lowest eigenpairs of `batch` Hamiltonians differing in V ([batch, nx, ny, nz]).
    X0 (optional, complex128): [batch, nb or nev, nx, ny, nz, 6]; X0 and
    psi_block, cheb_product, callback as in solve()."""
    V = _dev(V, torch.float64)
    if V.dim() != 4:
        raise ValueError("V must be [batch, nx, ny, nz]")
    batch = V.shape[0]
    shape = tuple(V.shape[1:])
    strain = _dev(strain, torch.float64)
    g = _grid(shape, h)
    ncomp = 3 if spin_free else 6
    X0d, xflags, nb = _x0(X0, (batch,), nev, nb, shape, ncomp)
    flags = (L.HKP_FLAG_GRAPH if graph else 0) | xflags | (L.HKP_FLAG_SPIN_FREE if spin_free else 0)
    if not polish:
        flags |= L.HKP_FLAG_NO_FP64_POLISH
    if not lock:
        flags |= L.HKP_FLAG_NO_LOCK
    if cheb_product:
        flags |= L.HKP_FLAG_CHEB_PRODUCT
    o = _opts(nev, nb, degree, max_iter, tol, precision, flags, seed)
    need = L.lib.hkp_workspace_bytes(C.byref(g), C.byref(o), batch)
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    npsi = _npsi(g, o, nev, return_psi and psi_block)
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    E = torch.empty((batch, nev), dtype=torch.float64, device="cuda")
    R = torch.empty((batch, nev), dtype=torch.float64, device="cuda")
    psi = torch.empty((batch, npsi) + shape + (ncomp,), dtype=torch.complex128, device="cuda") \
        if return_psi else None
    st = L.hkp_stats()
    mat = _material(material)
    s = _private_stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s), _iter_callback(callback):
        code = L.lib.hkp_solve_batch(C.byref(g), C.byref(mat), C.byref(o), batch, _ptr(V),
                                     _ptr(strain), _B(B), _ptr(X0d), _ptr(E), _ptr(psi), _ptr(R),
                                     _ptr(ws), C.c_size_t(ws.numel()), _stream(s),
                                     C.byref(st))
    torch.cuda.current_stream().wait_stream(s)
    L.check(code)
    return SolveResult(E, psi, R, st.as_dict(), code)


def solve_sweep(V, h, nev, strain=None, B=(0.0, 0.0, 0.0), nb=0, degree=0, tol=1e-8,
                precision="fp64", max_iter=200, seed=1, stride=8, graph=True, material=None,
                return_psi=False, polish=True, lock=True):
    """A sweep solved by continuation: the members 0, stride, 2 stride, ... in one
    batched solve from random blocks, then every other member in a second
    batched solve started from the nearest of those members' final blocks, guard
    vectors included (adjacent sweep points have close eigenvectors, so fewer
    filter passes are needed).  Same arguments and result layout as
    solve_batch."""
    V = _dev(V, torch.float64)
    if V.dim() != 4:
        raise ValueError("V must be [batch, nx, ny, nz]")
    if stride < 1:
        raise ValueError("stride must be >= 1")
    batch = V.shape[0]
    kw = dict(strain=strain, B=B, nb=nb, degree=degree, tol=tol, precision=precision,
              max_iter=max_iter, seed=seed, graph=graph, material=material, polish=polish,
              lock=lock)
    anchors = list(range(0, batch, stride))
    rest = [i for i in range(batch) if i % stride]
    ra = solve_batch(V[anchors], h, nev, return_psi=True, psi_block=True, **kw)
    E = torch.empty((batch, nev), dtype=torch.float64, device="cuda")
    R = torch.empty_like(E)
    psi = torch.empty((batch, nev) + ra.psi.shape[2:], dtype=torch.complex128, device="cuda") \
        if return_psi else None
    ia = torch.tensor(anchors, device="cuda")
    E[ia], R[ia] = ra.E, ra.resid
    if psi is not None:
        psi[ia] = ra.psi[:, :nev]
    stats = {"anchors": ra.stats}
    status = ra.status
    if rest:
        near = [min(round(i / stride), len(anchors) - 1) for i in rest]
        X0 = ra.psi[torch.tensor(near, device="cuda")]
        rr = solve_batch(V[rest], h, nev, X0=X0, return_psi=return_psi, **kw)
        ir = torch.tensor(rest, device="cuda")
        E[ir], R[ir] = rr.E, rr.resid
        if psi is not None:
            psi[ir] = rr.psi
        stats["rest"] = rr.stats
        status = max(status, rr.status)
    del ra
    return SolveResult(E, psi, R, stats, status)


def filter_step(V, h, X, Y_old=None, alpha=1.0, shift=0.0, beta=0.0, strain=None,
                B=(0.0, 0.0, 0.0), precision="fp64", material=None):
    """Y = alpha (H - shift) X + beta Y_old on a complex128 block [nvec, nx, ny, nz, 6]."""
    V = _dev(V, torch.float64)
    shape = tuple(V.shape)
    X = _dev(X, torch.complex128)
    nvec = X.shape[0]
    if tuple(X.shape[1:]) != shape + (6,):
        raise ValueError("X must be [nvec, nx, ny, nz, 6]")
    Y_old = _dev(Y_old, torch.complex128)
    strain = _dev(strain, torch.float64)
    g = _grid(shape, h)
    need = L.lib.hkp_apply_workspace_bytes(C.byref(g), nvec)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    Y = torch.empty_like(X)
    prec = L.HKP_PREC_MIXED if precision in ("mixed", 1) else L.HKP_PREC_FP64
    L.check(L.lib.hkp_filter_step(C.byref(g), C.byref(_material(material)), _ptr(V), _ptr(strain),
                                  _B(B), nvec, _ptr(X), _ptr(Y_old), _ptr(Y), float(alpha),
                                  float(shift), float(beta), prec, _ptr(ws),
                                  C.c_size_t(need), _stream()))
    return Y


def filter_step2(V, h, X, Y_old=None, alpha=(1.0, 1.0), shift=(0.0, 0.0), beta=(0.0, 0.0),
                 strain=None, B=(0.0, 0.0, 0.0), material=None):
    """Two Chebyshev steps in FP32 arithmetic: Y1 = alpha0 (H - shift0) X + beta0 Y_old,
    Y2 = alpha1 (H - shift1) Y1 + beta1 X on complex128 blocks [nvec, nx, ny, nz, 6].
    Returns (Y1, Y2, passes) with passes = 1 when one two-step pass did both."""
    V = _dev(V, torch.float64)
    shape = tuple(V.shape)
    X = _dev(X, torch.complex128)
    nvec = X.shape[0]
    if tuple(X.shape[1:]) != shape + (6,):
        raise ValueError("X must be [nvec, nx, ny, nz, 6]")
    Y_old = _dev(Y_old, torch.complex128)
    strain = _dev(strain, torch.float64)
    g = _grid(shape, h)
    need = L.lib.hkp_filter_step2_workspace_bytes(C.byref(g), nvec)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    Y1 = torch.empty_like(X)
    Y2 = torch.empty_like(X)
    two = lambda v: (C.c_double * 2)(*[float(x) for x in v])
    passes = C.c_int32(0)
    L.check(L.lib.hkp_filter_step2(C.byref(g), C.byref(_material(material)), _ptr(V),
                                   _ptr(strain), _B(B), nvec, _ptr(X), _ptr(Y_old), _ptr(Y1),
                                   _ptr(Y2), two(alpha), two(shift), two(beta), _ptr(ws),
                                   C.c_size_t(need), _stream(), C.byref(passes)))
    return Y1, Y2, int(passes.value)


def apply(V, h, X, strain=None, B=(0.0, 0.0, 0.0), precision="fp64", material=None):
    """Y = H X."""
    return filter_step(V, h, X, None, 1.0, 0.0, 0.0, strain, B, precision, material)


def gate_potential(V_bg, Lg, Vg):
    """V = V_bg + sum_g Vg[g] L[g] on the device."""
    V_bg = _dev(V_bg, torch.float64)
    Lg = _dev(Lg, torch.float64)
    Vg = _dev(Vg, torch.float64)
    out = torch.empty_like(V_bg)
    L.check(L.lib.hkp_gate_potential(V_bg.numel(), Lg.shape[0], _ptr(V_bg), _ptr(Lg), _ptr(Vg),
                                      _ptr(out), _stream()))
    return out


def hf_grad(psi, w, Lg):
    """grad[g] = sum_n w_n <psi_n| L_g |psi_n> (Hellmann-Feynman)."""
    psi = _dev(psi, torch.complex128)
    w = _dev(w, torch.float64)
    Lg = _dev(Lg, torch.float64)
    nev = psi.shape[0]
    N = Lg[0].numel()
    G = Lg.shape[0]
    need = L.lib.hkp_hf_grad_workspace_bytes(G)
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    grad = torch.empty(G, dtype=torch.float64, device="cuda")
    L.check(L.lib.hkp_hf_grad(N, nev, _ptr(psi), _ptr(w), G, _ptr(Lg), _ptr(grad), _ptr(ws),
                              C.c_size_t(need), _stream()))
    return grad


def soi_matrix(phi, delta_so=None, E=None, material=None):
    """[2M, 2M] spin-orbit matrix <phi_i s| H_SO |phi_j t> (index 2 i + s) of M
    spin-free orbitals phi [M, nx, ny, nz, 3] (from solve(..., spin_free=True));
    with E [M] the orbital energies go on the diagonal.  delta_so defaults to
    the material's."""
    phi = _dev(phi, torch.complex128)
    if phi.dim() != 5 or phi.shape[-1] != 3:
        raise ValueError("phi must be [M, nx, ny, nz, 3]")
    M = phi.shape[0]
    if delta_so is None:
        delta_so = _material(material).delta_so_eV
    g = _grid(tuple(phi.shape[1:4]), 1.0)
    need = L.lib.hkp_soi_workspace_bytes(C.byref(g), M)
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    E = _dev(E, torch.float64)
    out = torch.empty((2 * M, 2 * M), dtype=torch.complex128, device="cuda")
    L.check(L.lib.hkp_soi_matrix(C.byref(g), M, _ptr(phi), _ptr(E), float(delta_so), _ptr(out),
                                 _ptr(ws), C.c_size_t(need), _stream()))
    return out


@dataclass
class CIResult:
    E: torch.Tensor          # [K] two-hole energies, eV, ascending
    J: float                 # mean(E_1..E_3) - E_0, eV (nan if K < 4)
    vectors: torch.Tensor    # [K, K] complex (column k: state k) or None
    H: torch.Tensor          # [K, K] complex determinant matrix or None
    coulomb: torch.Tensor    # [M, M, M, M] complex (ik|jl) or None
    stats: dict
    status: int


def ci_solve(phi, E, h, pshape, offset, eps_r, dirichlet, delta_so=None, material=None,
             cg_tol=1e-12, cg_max_iter=20000, return_vectors=False, return_matrix=False,
             return_coulomb=False):
    """Two-hole configuration interaction in the determinants of the spin-orbitals
    of M spin-free orbitals phi [M, nx, ny, nz, 3] (energies E [M]); the Coulomb
    interaction comes from the device's Poisson problem (box `pshape`, the grid at
    `offset`) with every electrode grounded."""
    phi = _dev(phi, torch.complex128)
    if phi.dim() != 5 or phi.shape[-1] != 3:
        raise ValueError("phi must be [M, nx, ny, nz, 3]")
    M = phi.shape[0]
    E = _dev(E, torch.float64)
    eps_r = _dev(eps_r, torch.float64)
    dirichlet = _dev(dirichlet, torch.uint8)
    if delta_so is None:
        delta_so = _material(material).delta_so_eV
    g = _grid(tuple(phi.shape[1:4]), h)
    pg = _pgrid(pshape, offset)
    need = L.lib.hkp_ci_workspace_bytes(C.byref(g), M, C.byref(pg))
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    K = M * (2 * M - 1)
    ev = torch.empty(K, dtype=torch.float64, device="cuda")
    J = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    vec = torch.empty((K, K), dtype=torch.complex128, device="cuda") if return_vectors else None
    Hm = torch.empty((K, K), dtype=torch.complex128, device="cuda") if return_matrix else None
    Cc = torch.empty((M,) * 4, dtype=torch.complex128, device="cuda") if return_coulomb else None
    st = L.hkp_ci_stats()
    code = L.lib.hkp_ci_solve(C.byref(g), M, _ptr(phi), _ptr(E), float(delta_so), C.byref(pg),
                              _ptr(eps_r), _ptr(dirichlet), float(cg_tol), int(cg_max_iter),
                              _ptr(ev), _ptr(vec), _ptr(Hm), _ptr(Cc), _ptr(J), _ptr(ws),
                              C.c_size_t(need), _stream(), C.byref(st))
    L.check(code)
    return CIResult(ev, float(J[0]), vec, Hm, Cc, st.as_dict(), code)


# ---------------------------------------------------------------------------
# g-matrices and the effective two-spin model
# ---------------------------------------------------------------------------
@dataclass
class GMatrixResult:
    g: object            # numpy [4, 3, 3]: bonding, antibonding, left, right (row = Pauli)
    g_sym: object        # numpy [4, 3, 3] symmetric g-tensors
    centre: object       # numpy [4, 3] centres of charge, nm about the box centre
    kramers: object      # numpy [4, 3] tr M_b / mu_B (zero for Kramers doublets)
    E: object            # numpy [4] <psi_i|H|psi_i>, eV
    delta: float         # antibonding - bonding, eV
    t: float             # |delta| / sqrt(2), eV
    d: float             # distance between the left and right centres, nm
    raw: torch.Tensor    # the device hkp_gmatrix_result (input of two_spin_model)


def g_matrices(psi, V, h, strain=None, material=None):
    """g-matrices of the bonding (psi[0:2]) and antibonding (psi[2:4]) Kramers doublets
    and of the dots' doublets they localise to; psi [4, nx, ny, nz, 6] from a B = 0 solve."""
    psi = _dev(psi, torch.complex128)
    V = _dev(V, torch.float64)
    S = _dev(strain, torch.float64)
    if psi.dim() != 5 or psi.shape[0] != 4 or psi.shape[-1] != 6 or \
            tuple(psi.shape[1:4]) != tuple(V.shape):
        raise ValueError("psi must be [4, nx, ny, nz, 6] on V's grid")
    g = _grid(tuple(V.shape), h)
    mat = _material(material)
    need = L.lib.hkp_gmatrix_workspace_bytes(C.byref(g))
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    raw = torch.empty(C.sizeof(L.hkp_gmatrix_result) // 8, dtype=torch.float64, device="cuda")
    L.check(L.lib.hkp_gmatrix(C.byref(g), C.byref(mat), _ptr(V), _ptr(S), _ptr(psi), _ptr(raw),
                              _ptr(ws), C.c_size_t(need), _stream()))
    r = L.hkp_gmatrix_result.from_buffer_copy(raw.cpu().numpy().tobytes())
    import numpy as np
    return GMatrixResult(np.array(r.g).reshape(4, 3, 3), np.array(r.g_sym).reshape(4, 3, 3),
                         np.array(r.centre_nm).reshape(4, 3), np.array(r.kramers).reshape(4, 3),
                         np.array(r.E_eV), r.delta_eV, r.t_eV, r.d_nm, raw)


def two_spin_model(gm, J, B, n_so, lambda_so, d=0.0, return_matrix=False):
    """Eq. HB and the anisotropic exchange for every field in B [nB, 3] (tesla), from
    the left/right g-tensors and t of g_matrices(); J (eV, float or device [1]) is the
    exchange at the detuning of interest; d <= 0 takes the dots' distance from gm."""
    raw = gm.raw if isinstance(gm, GMatrixResult) else gm
    Bt = _dev(B, torch.float64).reshape(-1, 3)
    nB = Bt.shape[0]
    Jt = J if torch.is_tensor(J) else torch.tensor([float(J)], dtype=torch.float64)
    Jt = _dev(Jt, torch.float64).reshape(1)
    o = L.hkp_st_opts((C.c_double * 3)(*[float(v) for v in n_so]), float(lambda_so), float(d))
    width = C.sizeof(L.hkp_st_point) // 8
    pts = torch.empty((nB, width), dtype=torch.float64, device="cuda")
    H = torch.empty((nB, 5, 5), dtype=torch.complex128, device="cuda") if return_matrix else None
    L.check(L.lib.hkp_st_model(_ptr(raw), _ptr(Jt), C.byref(o), int(nB), _ptr(Bt), _ptr(pts),
                               _ptr(H), _stream()))
    return {"bbar": pts[:, 0:3], "db": pts[:, 3:6], "dEz": pts[:, 6], "E": pts[:, 7:12],
            "Jt": pts[:, 12:21].reshape(nB, 3, 3), "J_perp": pts[:, 21], "J_par": pts[:, 22],
            "H": H}


# ---------------------------------------------------------------------------
# self-consistent Schroedinger-Poisson loop
# ---------------------------------------------------------------------------
def _pgrid(pshape, offset=(0, 0, 0)):
    px, py, pz = (int(v) for v in pshape)
    ox, oy, oz = (int(v) for v in offset)
    return L.hkp_pgrid(px, py, pz, ox, oy, oz)


def poisson_preconditioner(kind):
    """Preconditioner of the Poisson CG solves that follow in this process:
    "multigrid" (default) or "jacobi".  Returns the previous one."""
    code = {"multigrid": L.HKP_PRECOND_MULTIGRID, "jacobi": L.HKP_PRECOND_JACOBI}.get(kind)
    if code is None:
        raise ValueError("kind must be 'multigrid' or 'jacobi'")
    prev = L.lib.hkp_poisson_preconditioner(code)
    L.check(min(prev, 0))
    return "multigrid" if prev == L.HKP_PRECOND_MULTIGRID else "jacobi"


def poisson(eps_r, dirichlet, phi_fixed, rho, h, phi0=None, tol=1e-12, max_iter=20000,
            graph=True):
    """phi (V) on the Poisson box [px, py, pz] from -div(eps_r grad phi) = (e/eps0) rho
    (rho in e/nm^3, may be None), electrode nodes (dirichlet != 0) at phi_fixed.
    graph: run on a private stream, where the library replays its CG iterations
    as a recorded hipGraph.  Returns (phi, cg_iterations, final |r|/|b|, status)."""
    eps_r = _dev(eps_r, torch.float64)
    shape = tuple(eps_r.shape)
    dirichlet = _dev(dirichlet, torch.uint8)
    phi_fixed = _dev(phi_fixed, torch.float64)
    rho = _dev(rho, torch.float64)
    for t in (dirichlet, phi_fixed) + ((rho,) if rho is not None else ()):
        if tuple(t.shape) != shape:
            raise ValueError("eps_r, dirichlet, phi_fixed and rho must share one [px, py, pz] shape")
    pg = _pgrid(shape)
    need = L.lib.hkp_poisson_workspace_bytes(C.byref(pg))
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    phi = torch.zeros(shape, dtype=torch.float64, device="cuda") if phi0 is None \
        else _dev(phi0, torch.float64).clone()
    it = C.c_int32(0)
    rel = C.c_double(0.0)
    args = (C.byref(pg), float(h), _ptr(eps_r), _ptr(dirichlet), _ptr(phi_fixed), _ptr(rho),
            _ptr(phi), float(tol), int(max_iter), _ptr(ws), C.c_size_t(need))
    if graph:
        s = _private_stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            code = L.lib.hkp_poisson(*args, _stream(s), C.byref(it), C.byref(rel))
        torch.cuda.current_stream().wait_stream(s)
    else:
        code = L.lib.hkp_poisson(*args, _stream(), C.byref(it), C.byref(rel))
    L.check(code)
    return phi, it.value, rel.value, code


def occupancy(E, n_holes, T):
    """Fermi-Dirac occupations of the hole levels E (eV) holding n_holes at T (K):
    returns (f, mu) as device tensors."""
    E = _dev(E, torch.float64)
    f = torch.empty_like(E)
    mu = torch.empty(1, dtype=torch.float64, device="cuda")
    L.check(L.lib.hkp_occupancy(E.numel(), _ptr(E), float(n_holes), float(T), _ptr(f), _ptr(mu),
                                _stream()))
    return f, mu[0]


def hole_density(psi, f, h):
    """sum_n f_n sum_c |psi_n,c|^2 / h^3 (nm^-3) for psi [nev, nx, ny, nz, 6]."""
    psi = _dev(psi, torch.complex128)
    f = _dev(f, torch.float64)
    shape = tuple(psi.shape[1:4])
    g = _grid(shape, h)
    out = torch.empty(shape, dtype=torch.float64, device="cuda")
    L.check(L.lib.hkp_hole_density(C.byref(g), psi.shape[0], _ptr(psi), _ptr(f), _ptr(out),
                                   _stream()))
    return out


@dataclass
class SPResult:
    phi: torch.Tensor        # [px, py, pz] V, the potential of the returned eigenpairs
    E: torch.Tensor          # [nev] eV
    psi: torch.Tensor        # [nev, nx, ny, nz, 6] or None
    resid: torch.Tensor      # [nev] eV
    density: torch.Tensor    # [nx, ny, nz] nm^-3
    stats: dict
    status: int


def sp_solve(V_off, h, nev, pshape, offset, eps_r, dirichlet, phi_fixed, n_holes, T,
             strain=None, B=(0.0, 0.0, 0.0), rho_fixed=None, phi0=None, nb=0, degree=0,
             tol=1e-8, precision="fp64", max_iter=200, seed=1, graph=False, material=None,
             mixing=0.3, history=5, tol_V=1e-8, sp_max_iter=100, cg_tol=1e-12,
             cg_max_iter=20000, return_psi=True, exact_eig=False, anneal_T=0.0,
             cheb_product=True):
    """Self-consistent Schroedinger-Poisson loop: V_off [nx, ny, nz] (eV) at `offset`
    inside the Poisson box `pshape`; eps_r, dirichlet, phi_fixed (and rho_fixed)
    on the box.  phi0: start from this potential instead of the hole-free one.
    exact_eig: every eigensolve to `tol` (default: looser while the potential
    still moves, `tol` for the final pass).
    anneal_T: if above T, the loop first converges at this temperature and then
    goes on at T from that potential (0: off).
    cheb_product: the eigensolves evaluate their Chebyshev filter in product form
    (the default here: the same polynomial with a third fewer bytes per step; on
    the 256 x 48 x 48 fin the annealed loop takes 0.87 s against 1.03 s with the
    three-term recurrence, results within the loop's tolerances of each other)."""
    V_off = _dev(V_off, torch.float64)
    shape = tuple(V_off.shape)
    strain = _dev(strain, torch.float64)
    eps_r = _dev(eps_r, torch.float64)
    dirichlet = _dev(dirichlet, torch.uint8)
    phi_fixed = _dev(phi_fixed, torch.float64)
    rho_fixed = _dev(rho_fixed, torch.float64)
    pshape = tuple(int(v) for v in pshape)
    for t in (eps_r, dirichlet, phi_fixed) + ((rho_fixed,) if rho_fixed is not None else ()):
        if tuple(t.shape) != pshape:
            raise ValueError("box fields must be [px, py, pz]")
    g = _grid(shape, h)
    pg = _pgrid(pshape, offset)
    flags = (L.HKP_FLAG_GRAPH if graph else 0) | (L.HKP_FLAG_CHEB_PRODUCT if cheb_product else 0)
    o = _opts(nev, nb, degree, max_iter, tol, precision, flags, seed)
    sp = L.hkp_sp_opts(float(n_holes), float(T), float(mixing), int(history), int(sp_max_iter),
                       float(tol_V), float(cg_tol), int(cg_max_iter),
                       (L.HKP_SP_PHI0 if phi0 is not None else 0)
                       | (L.HKP_SP_EXACT_EIG if exact_eig else 0), float(anneal_T))
    need = L.lib.hkp_sp_workspace_bytes(C.byref(g), C.byref(o), C.byref(pg), C.byref(sp))
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    phi = torch.zeros(pshape, dtype=torch.float64, device="cuda") if phi0 is None \
        else _dev(phi0, torch.float64).clone()
    E = torch.empty(nev, dtype=torch.float64, device="cuda")
    R = torch.empty(nev, dtype=torch.float64, device="cuda")
    dens = torch.empty(shape, dtype=torch.float64, device="cuda")
    psi = torch.empty((nev,) + shape + (6,), dtype=torch.complex128, device="cuda") \
        if return_psi else None
    st = L.hkp_sp_stats()
    mat = _material(material)
    s = _private_stream() if graph else None
    if s is not None:
        s.wait_stream(torch.cuda.current_stream())
        ctx = torch.cuda.stream(s)
    else:
        ctx = None
    args = (C.byref(g), C.byref(mat), C.byref(o), C.byref(pg), C.byref(sp), _ptr(V_off),
            _ptr(strain), _B(B), _ptr(eps_r), _ptr(dirichlet), _ptr(phi_fixed), _ptr(rho_fixed),
            _ptr(phi), _ptr(E), _ptr(psi), _ptr(R), _ptr(dens), _ptr(ws), C.c_size_t(need))
    if ctx is not None:
        with ctx:
            code = L.lib.hkp_sp_solve(*args, _stream(s), C.byref(st))
        torch.cuda.current_stream().wait_stream(s)
    else:
        code = L.lib.hkp_sp_solve(*args, _stream(), C.byref(st))
    L.check(code)
    return SPResult(phi, E, psi, R, dens, st.as_dict(), code)


def autotune(shape, h, nb, precision="fp64", with_strain=True, with_field=True):
    g = _grid(shape, h)
    prec = L.HKP_PREC_MIXED if precision in ("mixed", 1) else L.HKP_PREC_FP64
    need = workspace_bytes(shape, h, max(1, nb - 1), nb=nb, precision=precision)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    t = L.hkp_tune()
    L.check(L.lib.hkp_autotune(C.byref(g), nb, prec, int(with_strain), int(with_field), _ptr(ws),
                               C.c_size_t(need), _stream(), C.byref(t)))
    return dict(tile_y=t.tile_y, vgroup=t.vgroup, dma=t.dma, us_per_step=t.us_per_step,
                gbps=t.gbps, two_step=(t.two_step_tx, t.two_step_ty),
                us_per_step_two=t.us_per_step_two)


def tuned_shape(shape, h, nb, precision="fp64", with_strain=True, with_field=True):
    """The launch shape a solve on this grid and block size would use (tuned,
    cached or default), without timing anything."""
    g = _grid(shape, h)
    prec = L.HKP_PREC_MIXED if precision in ("mixed", 1) else L.HKP_PREC_FP64
    t = L.hkp_tune()
    L.check(L.lib.hkp_tuned_shape(C.byref(g), nb, prec, int(with_strain), int(with_field),
                                  C.byref(t)))
    return dict(tile_y=t.tile_y, vgroup=t.vgroup, dma=t.dma,
                two_step=(t.two_step_tx, t.two_step_ty))


def tune_cache_save(path):
    """Write the autotuners' cached choices (launch shapes, block sizes) to `path`
    under this device's architecture; returns the number of entries."""
    rc = L.lib.hkp_tune_cache_save(os.fsencode(path))
    L.check(rc)
    return rc


def tune_cache_load(path):
    """Take the entries of a cache file written for this device's architecture;
    returns the number taken (0 for another architecture's file)."""
    rc = L.lib.hkp_tune_cache_load(os.fsencode(path))
    L.check(rc)
    return rc


def tune_cache_clear():
    L.lib.hkp_tune_cache_clear()


def autotune_block(V, h, nev, strain=None, B=(0.0, 0.0, 0.0), candidates=None, tol=1e-8,
                   precision="fp64", degree=0, max_iter=200, seed=1, material=None):
    """Pick the block size by timing one complete solve of this Hamiltonian per
    candidate (default: nev + 8, nev + 16, nev + 24, rounded up to 8, <= 64).
    The choice is cached per (grid, nev, precision): later solve() and
    solve_batch() calls with nb=0 use it.  Returns dict(nb=..., seconds={nb: s})."""
    V = _dev(V, torch.float64)
    shape = tuple(V.shape)
    strain = _dev(strain, torch.float64)
    g = _grid(shape, h)
    if candidates is None:
        candidates = sorted({min(64, (nev + d + 7) // 8 * 8) for d in (8, 16, 24)})
        candidates = [c for c in candidates if c > nev]
    cand = (C.c_int32 * len(candidates))(*[int(c) for c in candidates])
    o = _opts(nev, max(candidates), degree, max_iter, tol, precision, 0, seed)
    need = L.lib.hkp_workspace_bytes(C.byref(g), C.byref(o), 1)
    if need == 0:
        raise L.HkpError(L.HKP_E_ARG, L.lib.hkp_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    o.nb = 0
    nb_out = C.c_int32(0)
    secs = (C.c_double * len(candidates))()
    mat = _material(material)
    code = L.lib.hkp_autotune_block(C.byref(g), C.byref(mat), C.byref(o), _ptr(V), _ptr(strain),
                                    _B(B), cand, len(candidates), _ptr(ws), C.c_size_t(need),
                                    _stream(), C.byref(nb_out), secs)
    L.check(code)
    if code != L.HKP_OK:
        raise L.HkpError(code, L.lib.hkp_last_error().decode())
    return dict(nb=int(nb_out.value), seconds={int(c): float(t) for c, t in zip(candidates, secs)})


class EigvalsFromPotential(torch.autograd.Function):
    """Gate voltages -> lowest eigenvalues, with a Hellmann-Feynman backward.

    forward(Vg [G], L [G, nx, ny, nz], V_bg [nx, ny, nz], cfg) -> E [nev]
    cfg: dict(h, nev, strain, B, tol, ...) passed to solve().
    Backward: dLoss/dVg = hf_grad(psi, dLoss/dE, L).  Degenerate eigenvalues
    (Kramers pairs at B = 0) must carry equal upstream weights, else the
    gradient of the individual levels is not defined and this raises.
    """

    @staticmethod
    def forward(ctx, Vg, Lg, V_bg, cfg):
        V = gate_potential(V_bg, Lg, Vg)
        kw = dict(cfg)
        h = kw.pop("h")
        nev = kw.pop("nev")
        kw.pop("degenerate_tol", None)   # a backward setting, not a solve() argument
        res = solve(V, h, nev, **kw)
        if res.status != L.HKP_OK:
            raise L.HkpError(res.status, "eigensolver did not converge")
        ctx.save_for_backward(res.psi, Lg, res.E)
        ctx.degenerate_tol = cfg.get("degenerate_tol", 1e-9)
        return res.E.clone()

    @staticmethod
    def backward(ctx, gE):
        psi, Lg, E = ctx.saved_tensors
        w = gE.detach().to(torch.float64).contiguous()
        # members of a degenerate group must carry equal weights
        e = E.detach().cpu()
        wc = w.cpu()
        i = 0
        n = e.numel()
        while i < n:
            j = i + 1
            while j < n and abs(float(e[j] - e[i])) <= ctx.degenerate_tol:
                j += 1
            if j - i > 1 and float((wc[i:j] - wc[i]).abs().max()) > 1e-12 * max(1.0, float(wc[i:j].abs().max())):
                raise ValueError("unequal weights within a degenerate eigenvalue group: "
                                 "the gradient of an individual degenerate level is undefined")
            i = j
        g = hf_grad(psi, w, Lg.reshape(Lg.shape[0], -1))
        return g, None, None, None
