"""The seeded input generators are deterministic and hit their stated statistics."""

import numpy as np

from synth import smooth_field, workload
from synth.inputs import _rng, fin_potential


def test_deterministic():
    a = workload("fin_small")
    b = workload("fin_small")
    assert np.array_equal(a.V, b.V) and np.array_equal(a.strain, b.strain)
    c = workload("fin_small", seed=99)
    assert not np.array_equal(a.V, c.V)


def test_smooth_field_exact_sigma_and_zero_mean():
    f = smooth_field((30, 20, 10), 0.4, 3.0, 0.5e-3, _rng(7, 0))
    assert abs(f.std() - 0.5e-3) < 1e-15
    assert abs(f.mean()) < 1e-18


def test_fin_mask_and_strain_recipe():
    w = workload("fin_small")
    fin = fin_potential(w.shape, w.h)
    # 10 nm wide fin: |y - yc| <= 5 nm is inside
    y = (np.arange(w.ny) + 1.0) * w.h
    yc = (w.ny + 1) * w.h / 2
    inside = np.abs(y - yc) <= 5.0
    assert np.all(fin[:, inside, :] == 0.0) and np.all(fin[:, ~inside, :] == 4.5)
    assert abs(w.strain[..., 2].mean() + 0.003) < 1e-12
    for k in (0, 1, 3, 4, 5):
        assert abs(w.strain[..., k].std() - 1e-4) < 1e-15


def test_harmonic_workload_shape_and_scale():
    w = workload("harmonic_10x8x8")
    assert w.V.shape == (10, 8, 8) and w.strain is None and w.nev == 8
    assert 0 < w.V.max() < 0.01


def test_sweep_barrier_profile():
    # only the metadata, to keep the CPU suite light
    from synth.inputs import build
    w = build("sweep64_dqd_192x40x40", small_shape=(24, 8, 8))
    b = w.extra["barrier"]
    assert w.V.shape == (64, 24, 8, 8)
    assert np.all(np.abs(b - np.linspace(0.020, 0.060, 64)) < 3e-3)
