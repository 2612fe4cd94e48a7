"""The autotuners' cache file on the GPU: a tuned launch shape and block size
survive save, clear and load (the file is keyed by this device's
architecture), and a solve after loading uses them and still matches the
oracle."""

import numpy as np
import pytest

from oracle import SI_MATERIAL, Grid, hamiltonian_ls, lowest_arpack
from synth import workload

pytestmark = pytest.mark.gpu


def test_tune_cache_round_trip(tmp_path):
    import torch
    import paper_2607_08447_amd as hkp
    w = workload("fin_small")
    print(f"tune cache round trip on {w.shape}", flush=True)
    hkp.tune_cache_clear()
    tuned = hkp.autotune(w.shape, w.h, 24, "mixed")
    V = torch.from_numpy(w.V).cuda()
    S = torch.from_numpy(w.strain).cuda()
    blk = hkp.autotune_block(V, w.h, 12, strain=S, B=w.B, candidates=[16, 24], tol=1e-6,
                             precision="mixed")
    path = tmp_path / "tune.txt"
    n = hkp.tune_cache_save(str(path))
    assert n >= 2
    assert path.read_text().splitlines()[1].startswith("arch gfx950")
    hkp.tune_cache_clear()
    assert hkp.tune_cache_load(str(path)) == n
    got = hkp.tuned_shape(w.shape, w.h, 24, "mixed")
    assert (got["tile_y"], got["vgroup"], got["dma"]) == \
        (tuned["tile_y"], tuned["vgroup"], tuned["dma"])
    res = hkp.solve(V, w.h, 12, strain=S, B=w.B, nb=0, tol=1e-6, precision="mixed")
    assert res.status == 0 and res.stats["nb"] == blk["nb"]
    H = hamiltonian_ls(Grid(*w.shape, w.h), SI_MATERIAL, w.V, w.strain.reshape(-1, 6), w.B)
    E_ref, _ = lowest_arpack(H, 12, tol=1e-13)
    assert np.abs(res.E.cpu().numpy() - E_ref).max() <= 1e-6
    hkp.tune_cache_clear()
