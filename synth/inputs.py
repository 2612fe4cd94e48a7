"""Seeded synthetic workloads standing in for the paper's device fields.

The paper's fields come from a FinFET geometry, a thermal-strain simulation and
a self-consistent Poisson solution that are not available; these generators
produce fields with the same kind of structure (a Si fin inside a 4.5 eV oxide
step, Gaussian gate footprints forming one or two dots, compressive uniaxial
strain with a smooth random perturbation, an in-plane magnetic field).

Recipe (all randomness from numpy PCG64 seeded per workload and per field):
  * smooth random field: white Gaussian noise -> Gaussian filter of standard
    deviation ell/h grid cells (reflecting edges) -> mean removed -> rescaled to
    the exact sample standard deviation sigma.
  * gate footprint: Gaussian along x with FWHM 8 nm, uniform in y and z.
  * fin: |y - y_c| <= 5 nm and |z - z_c| <= 10 nm (clipped to the box); the
    potential is raised by 4.5 eV outside.
  * strain: e_zz = -0.003 everywhere plus a smooth perturbation of sigma 1e-4
    (ell = 4 nm) on each Voigt component (xx, yy, zz, yz, xz, xy).
  * harmonic well: V = (hbar w)^2 |r - r0|^2 / (4 g1 E0), the isotropic
    oscillator of mass m0/g1 with level spacing hbar w.

Units: eV, nm, T.  Arrays are C-ordered [nx][ny][nz] (x slowest), Voigt last.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy.ndimage import gaussian_filter

# constants of the input recipe (harmonic well only)
_E0 = 0.03809982116     # hbar^2/(2 m0), eV nm^2
_GAMMA1 = 4.285         # Si, Table I
_FWHM_TO_SIGMA = 1.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)))


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    V: np.ndarray                       # [nx,ny,nz] or [batch,nx,ny,nz], eV
    strain: Optional[np.ndarray]        # [nx,ny,nz,6] or None
    B: tuple                            # Tesla
    nev: int
    nb: int                             # suggested block size
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def npts(self):
        return self.nx * self.ny * self.nz

    @property
    def batch(self):
        return self.V.shape[0] if self.V.ndim == 4 else 1


def _rng(seed, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def coords(shape, h):
    nx, ny, nz = shape
    x = (np.arange(nx) + 1.0) * h
    y = (np.arange(ny) + 1.0) * h
    z = (np.arange(nz) + 1.0) * h
    centre = np.array([(nx + 1) * h / 2, (ny + 1) * h / 2, (nz + 1) * h / 2])
    return x, y, z, centre


def smooth_field(shape, h, ell, sigma, rng):
    """Gaussian-filtered white noise with exact sample std sigma and zero mean."""
    w = rng.standard_normal(shape)
    s = gaussian_filter(w, sigma=ell / h, mode="reflect")
    s = s - s.mean()
    sd = s.std()
    return s * (sigma / sd) if sd > 0 else s


def gaussian_gate(x, xg, fwhm=8.0):
    sg = fwhm * _FWHM_TO_SIGMA
    return np.exp(-0.5 * ((x - xg) / sg) ** 2)


def fin_potential(shape, h, oxide=4.5, half_width_y=5.0, half_height_z=10.0):
    nx, ny, nz = shape
    _, y, z, c = coords(shape, h)
    out_y = np.abs(y - c[1]) > half_width_y
    out_z = np.abs(z - c[2]) > half_height_z
    mask = out_y[:, None] | out_z[None, :]
    return np.broadcast_to(np.where(mask, oxide, 0.0)[None, :, :], shape).copy()


def strain_field(shape, h, rng, ezz=-0.003, sigma=1e-4, ell=4.0):
    e = np.zeros(tuple(shape) + (6,))
    for k in range(6):
        e[..., k] = smooth_field(shape, h, ell, sigma, rng)
    e[..., 2] += ezz
    return e


def random_block(shape_or_n, nvec, seed, stream=99):
    """Seeded complex Gaussian block (nvec, n) for operator-level parity tests."""
    n = int(np.prod(shape_or_n)) if np.ndim(shape_or_n) else int(shape_or_n)
    r = _rng(seed, stream)
    return (r.standard_normal((nvec, n)) + 1j * r.standard_normal((nvec, n)))


def _harmonic(seed=1, shape=(10, 8, 8), h=0.5, hw=0.002, sigma=0.5e-3, ell=1.0):
    x, y, z, c = coords(shape, h)
    r2 = ((x - c[0]) ** 2)[:, None, None] + ((y - c[1]) ** 2)[None, :, None] \
        + ((z - c[2]) ** 2)[None, None, :]
    V = hw ** 2 * r2 / (4.0 * _GAMMA1 * _E0)
    V = V + smooth_field(shape, h, ell, sigma, _rng(seed, 0))
    return V


def _gates_1d(x, centres, amps):
    v = np.zeros_like(x)
    for xg, a in zip(centres, amps):
        v = v + a * gaussian_gate(x, xg)
    return v


def _dqd_x_profile(x, xc, plunger=-0.040, barrier=0.030, sep=30.0):
    return _gates_1d(x, [xc - sep / 2, xc + sep / 2, xc], [plunger, plunger, barrier])


def build(name, seed=None, small_shape=None):
    """Construct a named workload.  `small_shape` rescales the fin/DQD recipes to
    another grid (used by parity tests on grids the CPU oracle can handle)."""
    if name == "harmonic_10x8x8":
        s = 1 if seed is None else seed
        shape = (10, 8, 8) if small_shape is None else small_shape
        V = _harmonic(s, shape)
        return Workload(name, *shape, 0.5, V, None, (0.0, 0.0, 0.0), 8, 16)
    if name in ("fin_qd_128x40x40", "dqd_256x48x48", "sweep64_dqd_192x40x40",
                "adjoint_dqd_192x40x40", "fin_small", "dqd_small"):
        defaults = {
            "fin_qd_128x40x40": ((128, 40, 40), 2),
            "dqd_256x48x48": ((256, 48, 48), 3),
            "sweep64_dqd_192x40x40": ((192, 40, 40), 4),
            "adjoint_dqd_192x40x40": ((192, 40, 40), 5),
            "fin_small": ((40, 14, 12), 11),
            "dqd_small": ((64, 12, 10), 12),
        }
        shape, s0 = defaults[name]
        s = s0 if seed is None else seed
        if small_shape is not None:
            shape = tuple(small_shape)
        h = 0.4
        x, y, z, c = coords(shape, h)
        fin = fin_potential(shape, h)
        strain = strain_field(shape, h, _rng(s, 1))
        B = (0.5, 0.0, 0.0)
        if name in ("fin_qd_128x40x40", "fin_small"):
            r = _rng(s, 2)
            amps = -r.uniform(0.010, 0.060, size=5)
            L = x[-1] - x[0]
            centres = c[0] + np.linspace(-0.4, 0.4, 5) * L
            V = fin + _gates_1d(x, centres, amps)[:, None, None]
            return Workload(name, *shape, h, V, strain, B, 16, 32,
                            extra=dict(gate_amps=amps, gate_centres=centres))
        if name in ("dqd_256x48x48", "dqd_small"):
            V = fin + _dqd_x_profile(x, c[0])[:, None, None]
            return Workload(name, *shape, h, V, strain, B, 32, 48)
        if name == "sweep64_dqd_192x40x40":
            r = _rng(s, 3)
            nb_ham = 64
            barrier = np.linspace(0.020, 0.060, nb_ham) + r.normal(0.0, 0.5e-3, nb_ham)
            Vs = np.empty((nb_ham,) + tuple(shape))
            for i in range(nb_ham):
                Vs[i] = fin + _dqd_x_profile(x, c[0], barrier=barrier[i])[:, None, None]
            return Workload(name, *shape, h, Vs, strain, B, 16, 24,
                            extra=dict(barrier=barrier))
        if name == "adjoint_dqd_192x40x40":
            r = _rng(s, 4)
            centres = np.array([c[0] - 30.0, c[0] - 15.0, c[0], c[0] + 15.0, c[0] + 30.0])
            alpha = r.uniform(0.05, 0.3, size=5)
            Lg = np.stack([np.broadcast_to((a * gaussian_gate(x, xg))[:, None, None], shape)
                           for a, xg in zip(alpha, centres)]).copy()
            V_bg = fin + _dqd_x_profile(x, c[0])[:, None, None]
            return Workload(name, *shape, h, V_bg, strain, (0.0, 0.0, 0.0), 8, 16,
                            extra=dict(L=Lg, alpha=alpha, centres=centres,
                                       Vg0=np.zeros(5)))
    raise KeyError(name)


WORKLOADS = ("harmonic_10x8x8", "fin_qd_128x40x40", "dqd_256x48x48",
             "sweep64_dqd_192x40x40", "adjoint_dqd_192x40x40")


def workload(name, **kw):
    return build(name, **kw)


# ---------------------------------------------------------------------------
# Self-consistent Schroedinger-Poisson devices
# ---------------------------------------------------------------------------
@dataclass
class SPDevice:
    """A gated fin for the self-consistent loop: the Schroedinger grid (shape, h)
    sits at `offset` inside the Poisson box `pshape` (same spacing)."""
    name: str
    shape: tuple
    h: float
    pshape: tuple
    offset: tuple
    V_off: np.ndarray          # [nx,ny,nz] band offset (oxide step), eV
    strain: Optional[np.ndarray]
    B: tuple
    eps_r: np.ndarray          # [px,py,pz]
    dirichlet: np.ndarray      # [px,py,pz] uint8, 1 = electrode node
    phi_fixed: np.ndarray      # [px,py,pz] electrode potentials (V), 0 elsewhere
    n_holes: float
    T: float
    nev: int
    nb: int
    gates: dict = field(default_factory=dict)


def sp_device(name):
    """Recipe: the fin of the other workloads (4.5 eV oxide step outside a 10 x 20 nm
    cross-section) with its Schroedinger grid padded on every side inside the
    Poisson box; eps_r = 11.7 (Si) where V_off = 0 and 3.9 (SiO2) elsewhere.
    Electrodes: the bottom face of the box is a grounded substrate contact; on the
    top face, strips across y of 10 nm along x: two plungers at x_c -+ 15 nm and a
    barrier gate at x_c (these Dirichlet patches are the gates of Fig. 1, with
    the rest of every outer face field-free).  Two holes at 1.5 K (Sec. II.C)."""
    cfg = {
        # name: (S shape, pad (x, y, z-below, z-above), gate volts (plunger, barrier),
        #        strain, B, nev, nb)
        "sp_tiny": ((12, 6, 6), (2, 2, 2, 3), (-0.30, -0.05), False, (0.0, 0.0, 0.0), 8, 16),
        "sp_dqd_small": ((24, 8, 8), (3, 3, 2, 4), (-0.30, -0.05), False, (0.0, 0.0, 0.0),
                         8, 16),
        "sp_dqd_256x48x48": ((256, 48, 48), (8, 8, 16, 24), (-0.30, -0.05), True,
                             (0.5, 0.0, 0.0), 8, 16),
    }
    if name not in cfg:
        raise KeyError(name)
    shape, pad, (vp, vb), with_strain, B, nev, nb = cfg[name]
    h = 0.4
    px_, py_, pzb, pza = pad
    pshape = (shape[0] + 2 * px_, shape[1] + 2 * py_, shape[2] + pzb + pza)
    offset = (px_, py_, pzb)
    V_off = fin_potential(shape, h)
    eps = np.full(pshape, 3.9)
    ox, oy, oz = offset
    eps[ox:ox + shape[0], oy:oy + shape[1], oz:oz + shape[2]] = np.where(V_off == 0.0, 11.7,
                                                                         3.9)
    dirichlet = np.zeros(pshape, dtype=np.uint8)
    phi_fixed = np.zeros(pshape)
    dirichlet[:, :, 0] = 1                              # substrate contact, 0 V
    xP = (np.arange(pshape[0]) + 1.0) * h
    xc = (ox + (shape[0] + 1) / 2.0) * h                # fin centre in box coordinates
    strips = {"P1": (xc - 15.0, vp), "B": (xc, vb), "P2": (xc + 15.0, vp)}
    if shape[0] * h < 40.0:                             # short fins: one plunger, centred
        strips = {"P1": (xc, vp)}
    for xg, v in strips.values():
        on = np.abs(xP - xg) <= 5.0 + 1e-6 * h          # edges on a node count (both sides)
        dirichlet[on, :, -1] = 1
        phi_fixed[on, :, -1] = v
    strain = strain_field(shape, h, _rng(21, 1)) if with_strain else None
    return SPDevice(name, shape, h, pshape, offset, V_off, strain, B, eps, dirichlet,
                    phi_fixed, 2.0, 1.5, nev, nb, gates=strips)
