"""The allocation-free Hellmann-Feynman entry point (hkp_hf_grad_noalloc, block
partial sums in a static device array) against hkp_hf_grad with a caller
workspace, through the C ABI: two calls in a row, the second smaller, and the
oracle's gradient formula for both."""

import ctypes as C

import numpy as np
import pytest

from oracle import hf_gradient

pytestmark = pytest.mark.gpu


def _case(rng, shape, nev, G):
    N = int(np.prod(shape))
    psi = rng.standard_normal((nev, N * 6)) + 1j * rng.standard_normal((nev, N * 6))
    return N, psi, rng.random(nev), rng.random((G, N))


def _grads(L, torch, N, psi, w, Lg):
    nev, G = psi.shape[0], Lg.shape[0]
    psi_d = torch.from_numpy(psi).cuda()
    w_d = torch.from_numpy(w).cuda()
    L_d = torch.from_numpy(Lg).cuda()
    g_ws = torch.full((G,), float("nan"), dtype=torch.float64, device="cuda")
    g_na = torch.full((G,), float("nan"), dtype=torch.float64, device="cuda")
    need = L.lib.hkp_hf_grad_workspace_bytes(G)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: C.c_void_p(t.data_ptr())
    assert L.lib.hkp_hf_grad(N, nev, P(psi_d), P(w_d), G, P(L_d), P(g_ws), P(ws),
                             C.c_size_t(need), s) == L.HKP_OK
    assert L.lib.hkp_hf_grad_noalloc(N, nev, P(psi_d), P(w_d), G, P(L_d), P(g_na), s) == L.HKP_OK
    torch.cuda.synchronize()
    return g_ws.cpu().numpy(), g_na.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice():
    import torch
    from paper_2607_08447_amd import _lib as L
    print("no-alloc HF gradient: 2 calls (30x9x7, nev 8, G 16; then 11x5x3, nev 3, G 3)",
          flush=True)
    rng = np.random.default_rng(11)
    for shape, nev, G in (((30, 9, 7), 8, 16), ((11, 5, 3), 3, 3)):
        N, psi, w, Lg = _case(rng, shape, nev, G)
        g_ws, g_na = _grads(L, torch, N, psi, w, Lg)
        # the same kernels in the same fixed reduction order: identical results
        assert np.array_equal(g_na, g_ws), (g_na, g_ws)
        ref = hf_gradient(psi.T, w, Lg)
        assert np.abs(g_na - ref).max() <= 1e-13 * np.abs(ref).max()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_2607_08447_amd import _lib as L
    fake = C.c_void_p(0x1000)
    for G in (0, 17):
        assert L.lib.hkp_hf_grad_noalloc(100, 2, fake, fake, G, fake, fake, None) == L.HKP_E_ARG
    assert b"16" in L.lib.hkp_last_error()
    assert L.lib.hkp_hf_grad_noalloc(0, 2, fake, fake, 4, fake, fake, None) == L.HKP_E_ARG
