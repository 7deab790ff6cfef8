"""Unit helpers for inputs given the way the paper's programs take them.

turbo_eels takes q1, q2, q3 in units of 2 pi / a (a = celldm(1) in bohr) and
turbo_spectrum takes the broadening epsil in Rydberg (Sec. 3.2-3.3, App. A);
the library works in Hartree atomic units throughout.
"""
import math

BOHR_IN_ANGSTROM = 0.529177210903   # CODATA 2018
HARTREE_IN_RY = 2.0


def q_from_alat_units(q_2pi_over_a, alat_bohr):
    """Cartesian q in bohr^-1 from components in units of 2 pi / a."""
    return [2.0 * math.pi / alat_bohr * float(c) for c in q_2pi_over_a]


def inv_bohr_to_inv_angstrom(x):
    return x / BOHR_IN_ANGSTROM


def ry_to_ha(x):
    return x / HARTREE_IN_RY
