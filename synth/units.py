"""Unit conversion used to turn spring constants into frequencies (input side only).

Frequencies are in rad/ps for force constants in eV/Angstrom^2 and masses in amu:
omega = OMEGA_UNIT * sqrt(eigenvalue of D), OMEGA_UNIT = sqrt(eV / (Angstrom^2 amu)) in rad/ps.
"""
import math

_EV = 1.602176634e-19          # J (exact, SI 2019)
_AMU = 1.66053906660e-27       # kg (CODATA 2018)
_ANGSTROM = 1.0e-10            # m

OMEGA_UNIT = math.sqrt(_EV / (_ANGSTROM**2 * _AMU)) * 1.0e-12   # rad/ps
