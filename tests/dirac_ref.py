"""Closed-form hydrogenic Dirac-Coulomb energies (textbook), used as pins."""
import math


def dirac_energy(Z: float, n: int, kappa: int, c: float) -> float:
    """Bound-state energy minus the rest energy, in Hartree, for a point
    nucleus:  E = c^2 ([1 + (Z/c)^2 / (n - |k| + sqrt(k^2 - (Z/c)^2))^2]^(-1/2) - 1)."""
    za = Z / c
    k = abs(kappa)
    denom = n - k + math.sqrt(k * k - za * za)
    return c * c * ((1.0 + (za / denom) ** 2) ** -0.5 - 1.0)


def dirac_1s(Z: float, c: float) -> float:
    """c^2 (sqrt(1 - (Z/c)^2) - 1), written without cancellation."""
    za2 = (Z / c) ** 2
    return -c * c * za2 / (1.0 + math.sqrt(1.0 - za2))
