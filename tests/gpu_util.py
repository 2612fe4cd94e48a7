"""Helpers shared by the GPU tests (no arithmetic of the method)."""

import numpy as np


def abi_block(X):
    """(nvec, 6N) oracle-ordered complex block -> ABI layout [nvec][nx][ny][nz][6]
    (identical memory order: point index (x ny + y) nz + z, component fastest)."""
    return X


def to_numpy(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
