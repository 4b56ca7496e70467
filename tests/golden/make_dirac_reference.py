"""Writes dirac_reference.txt from the closed-form Dirac-Coulomb formula."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from tests.dirac_ref import dirac_energy  # noqa: E402

C = 137.035999084
LEVELS = [(10, 1, -1), (47, 1, -1), (47, 2, -1), (47, 2, 1), (47, 2, -2), (17, 1, -1), (79, 1, -1)]

if __name__ == "__main__":
    lines = ["# Hydrogenic Dirac-Coulomb energies (point nucleus) used by the oracle pins.",
             "# E(n, kappa) = c^2 ( [1 + (Z/c)^2 / (n - |kappa| + sqrt(kappa^2 - (Z/c)^2))^2]^(-1/2) - 1 )",
             "# c = 137.035999084 a.u.; values written by tests/golden/make_dirac_reference.py",
             "# Z  n  kappa  E/Eh"]
    for Z, n, k in LEVELS:
        lines.append(f"{Z} {n} {k} {dirac_energy(Z, n, k, C):.12f}")
    open(os.path.join(HERE, "dirac_reference.txt"), "w").write("\n".join(lines) + "\n")
