"""Pins of the unit constants and the material parameters (CPU only).

The unit constants are derived here from the CODATA 2018 SI values, which
is independent of the literals the oracle and the library carry: each
literal must equal the derived value rounded to its ten significant digits,
so a changed digit fails.  The material values are compared with the
literals printed in Table I (Appendix A); gamma3 is the one reading that
departs from the table (1.446 instead of 1.21), fixed by the workloads.
"""

import ctypes as C
import math

import pytest

import oracle
from oracle import E0, E_OVER_HBAR, MU_B, SI_MATERIAL

# CODATA 2018: h and e exact in the SI, m0 measured
H_PLANCK = 6.62607015e-34       # J s
E_CHARGE = 1.602176634e-19      # C
M_ELECTRON = 9.1093837015e-31   # kg
HBAR = H_PLANCK / (2.0 * math.pi)

DERIVED = {
    # hbar^2 / (2 m0): J m^2 -> eV nm^2
    "E0": HBAR ** 2 / (2.0 * M_ELECTRON) / E_CHARGE * 1e18,
    # mu_B = e hbar / (2 m0): J/T -> eV/T
    "MU_B": E_CHARGE * HBAR / (2.0 * M_ELECTRON) / E_CHARGE,
    # e / hbar: 1/(T m^2) -> 1/(T nm^2)
    "E_OVER_HBAR": E_CHARGE / HBAR * 1e-18,
}

# Table I (Appendix A), Si row: gamma1..3, Delta_0 (eV), kappa, a_v, b, d (eV)
TABLE_I = dict(gamma1=4.285, gamma2=0.339, gamma3=1.21, delta_so=0.044, kappa=-0.42,
               a_v=2.46, b=-2.35, d=-5.32)
GAMMA3_WORKLOAD = 1.446


def _ten_digits(x):
    return float(f"{x:.9e}")


def test_derived_constants_match_textbook_values():
    # the derivation itself, against independently known approximate values
    assert abs(DERIVED["E0"] - 0.0381) < 1e-5           # 3.81 eV A^2
    assert abs(DERIVED["MU_B"] - 5.788e-5) < 1e-8
    assert abs(DERIVED["E_OVER_HBAR"] - 1.5193e-3) < 1e-7


@pytest.mark.parametrize("name,value", [("E0", E0), ("MU_B", MU_B),
                                        ("E_OVER_HBAR", E_OVER_HBAR)])
def test_oracle_unit_constants(name, value):
    assert value == _ten_digits(DERIVED[name]), (name, value, DERIVED[name])
    assert abs(value / DERIVED[name] - 1.0) < 1e-9


def test_library_unit_constants():
    from paper_2607_08447_amd import _lib as L
    out = (C.c_double * 3)()
    L.lib.hkp_unit_constants(out)
    for k, name in enumerate(("E0", "MU_B", "E_OVER_HBAR")):
        assert out[k] == _ten_digits(DERIVED[name]), (name, out[k])


def test_oracle_material_is_table_one():
    for k, v in TABLE_I.items():
        want = GAMMA3_WORKLOAD if k == "gamma3" else v
        assert SI_MATERIAL[k] == want, k
    assert set(SI_MATERIAL) == set(TABLE_I)


def test_library_default_material_is_table_one():
    from paper_2607_08447_amd import _lib as L
    m = L.hkp_material()
    L.lib.hkp_default_material(C.byref(m))
    got = dict(gamma1=m.gamma1, gamma2=m.gamma2, gamma3=m.gamma3, delta_so=m.delta_so_eV,
               kappa=m.kappa, a_v=m.a_v_eV, b=m.b_eV, d=m.d_eV)
    for k, v in TABLE_I.items():
        want = GAMMA3_WORKLOAD if k == "gamma3" else v
        assert got[k] == want, k


def test_oracle_exports():
    assert oracle.E0 is E0 and oracle.MU_B is MU_B and oracle.E_OVER_HBAR is E_OVER_HBAR
