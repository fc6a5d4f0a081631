"""Physical-unit helper: the couplings of Eq. (S.4) from atom numbers and
scattering lengths.

With the oscillator length l0 = sqrt(hbar / (m omega)) of the in-plane trap
and the trap aspect ratio kappa = omega_z / omega, the quasi-2D couplings are

    c0 = 2 N sqrt(2 pi kappa) (a0 + 2 a2) / (3 l0)
    c2 = 2 N sqrt(2 pi kappa) (a2 - a0) / (3 l0)

(a0, a2: s-wave scattering lengths in the total-spin 0 and 2 channels).
"""
import math

BOHR_M = 5.29177210903e-11  # CODATA 2018 Bohr radius, metres
HBAR = 1.054571817e-34      # J s


def oscillator_length(mass_kg: float, omega_rad_s: float) -> float:
    """l0 = sqrt(hbar / (m omega)) in metres."""
    return math.sqrt(HBAR / (mass_kg * omega_rad_s))


def couplings(n_atoms: float, a0_bohr: float, a2_bohr: float, l0_m: float, kappa: float = 1.0):
    """(c0, c2) of Eq. (S.4); scattering lengths in Bohr radii, l0 in metres."""
    if not (n_atoms > 0 and l0_m > 0 and kappa > 0):
        raise ValueError("n_atoms, l0_m and kappa must be positive")
    g = 2.0 * n_atoms * math.sqrt(2.0 * math.pi * kappa) / (3.0 * l0_m)
    return g * (a0_bohr + 2.0 * a2_bohr) * BOHR_M, g * (a2_bohr - a0_bohr) * BOHR_M
