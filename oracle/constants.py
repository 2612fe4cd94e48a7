"""Physical constants and the Si material of the paper (Appendix A, Table I).

Units throughout the oracle: energy eV, length nm, magnetic field T.
"""

# Unit constants from the CODATA 2018 SI values (h and e exact, m0 =
# 9.1093837015e-31 kg), each rounded to ten significant digits.
# hbar^2 / (2 m0) in eV nm^2
E0 = 0.03809982116
# Bohr magneton e hbar / (2 m0) in eV/T
MU_B = 5.788381806e-5
# e / hbar in 1/(T nm^2): the Peierls phase of a straight link is
# (e/hbar) * integral A . dl
E_OVER_HBAR = 1.519267448e-3

# Si parameters (Table I).  gamma3 is 1.446 here: Table I prints 1.21, the
# workload definition fixes 1.446; both are runtime parameters.
SI_MATERIAL = dict(
    gamma1=4.285, gamma2=0.339, gamma3=1.446,
    delta_so=0.044, kappa=-0.42,
    a_v=2.46, b=-2.35, d=-5.32,
)
