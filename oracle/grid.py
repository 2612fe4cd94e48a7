"""Finite-difference grid and the discrete kinetic operators (paper Sec. II.B).

The grid holds interior points r = ((i+1)h, (j+1)h, (k+1)h), 0 <= i < nx etc.
Hard wall (the paper's Dirichlet condition at the Si surface): psi = 0 on the
virtual layer one spacing outside the grid.  A periodic option exists only for
bulk-dispersion checks (B = 0).

Point index p = (i*ny + j)*nz + k  (x slowest, z fastest).

Magnetic field enters through Peierls link variables
    U_a(r) = exp(i (e/hbar) h A_a(r + h e_a / 2)),
exact for the linear vector potentials used here (midpoint rule on a linear
integrand).  The charge sign is that of the electron: k -> -i grad + (e/hbar) A.
"""

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .constants import E_OVER_HBAR


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    h: float
    periodic: bool = False

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def npts(self):
        return self.nx * self.ny * self.nz

    def coords(self):
        """Arrays x, y, z of shape (nx, ny, nz), in nm."""
        ix = (np.arange(self.nx) + 1.0) * self.h
        iy = (np.arange(self.ny) + 1.0) * self.h
        iz = (np.arange(self.nz) + 1.0) * self.h
        return np.meshgrid(ix, iy, iz, indexing="ij")

    def centre(self):
        return np.array([(self.nx + 1) * self.h / 2, (self.ny + 1) * self.h / 2,
                         (self.nz + 1) * self.h / 2])


def vector_potential(gauge, B, rel):
    """A(r) for r - r0 given as a tuple of arrays rel = (X, Y, Z).

    'symmetric':  A = B x (r - r0) / 2
    'landau':     A = (By Z - Bz Y, 0, Bx Y)     (curl A = B as well)
    """
    Bx, By, Bz = (float(b) for b in B)
    X, Y, Z = rel
    if gauge == "symmetric":
        return (0.5 * (By * Z - Bz * Y), 0.5 * (Bz * X - Bx * Z), 0.5 * (Bx * Y - By * X))
    if gauge == "landau":
        return (By * Z - Bz * Y, 0.0 * X, Bx * Y)
    raise ValueError(f"unknown gauge {gauge!r}")


def link_phases(grid, axis, B, gauge="symmetric", origin=None):
    """U_axis(r) for the link r -> r + h e_axis at every grid point (nx, ny, nz).

    origin: the gauge origin r0 as an offset (nm) from the box centre (None: the centre)."""
    x, y, z = grid.coords()
    r0 = grid.centre() + (0.0 if origin is None else np.asarray(origin, dtype=float))
    mid = [x - r0[0], y - r0[1], z - r0[2]]
    mid[axis] = mid[axis] + 0.5 * grid.h
    A = vector_potential(gauge, B, tuple(mid))
    return np.exp(1j * E_OVER_HBAR * grid.h * np.asarray(A[axis], dtype=float)
                  * np.ones(grid.shape))


def shift_operator(grid, axis, B=(0.0, 0.0, 0.0), gauge="symmetric", origin=None):
    """Sparse T_a with (T_a psi)(r) = U_a(r) psi(r + e_a); zero past a hard wall."""
    if grid.periodic and any(float(b) != 0.0 for b in B):
        raise ValueError("periodic grids are only supported at B = 0")
    n = grid.shape
    idx = np.arange(grid.npts).reshape(n)
    phase = link_phases(grid, axis, B, gauge, origin)
    if grid.periodic:
        rows = idx.ravel()
        cols = np.roll(idx, -1, axis=axis).ravel()
        vals = phase.ravel()
    else:
        sl_src = [slice(None)] * 3
        sl_dst = [slice(None)] * 3
        sl_src[axis] = slice(0, n[axis] - 1)
        sl_dst[axis] = slice(1, n[axis])
        rows = idx[tuple(sl_src)].ravel()
        cols = idx[tuple(sl_dst)].ravel()
        vals = phase[tuple(sl_src)].ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.npts, grid.npts))


def kinetic_operators(grid, B=(0.0, 0.0, 0.0), gauge="symmetric", origin=None):
    """The discrete k-operators of the finite-difference k.p Hamiltonian.

    Kaa[a]      = (2 - T_a - T_a^H) / h^2          (compact 3-point k_a^2)
    Ka[a]       = -i (T_a - T_a^H) / (2h)          (central k_a)
    Ksym[(a,b)] = (Ka Kb + Kb Ka) / 2              (symmetrised k_a k_b, a != b)
    All are Hermitian.  Ksym touches the four (a,b)-diagonal neighbours only.
    """
    h = grid.h
    eye = sp.identity(grid.npts, dtype=complex, format="csr")
    T = [shift_operator(grid, a, B, gauge, origin) for a in range(3)]
    Kaa = [((2.0 * eye - t - t.getH()) / h**2).tocsr() for t in T]
    Ka = [((-1j) * (t - t.getH()) / (2.0 * h)).tocsr() for t in T]
    Ksym = {}
    for a in range(3):
        for b in range(a + 1, 3):
            m = (0.5 * (Ka[a] @ Ka[b] + Ka[b] @ Ka[a])).tocsr()
            Ksym[(a, b)] = m
            Ksym[(b, a)] = m
    return Kaa, Ka, Ksym
