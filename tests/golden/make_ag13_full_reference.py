"""Writes ag13_full_seed0.npz: reference values of the full (non-local)
two-component X2C Hamiltonian of the coupled 13-atom silver molecule
(x2c_inputs.ag13_molecule(0): 2496 scalar functions, 4992 spinors, 4c
dimension 9984), computed by the CPU oracle only (oracle.x2c_direct and the
oracle's brute-force 4c spectrum, Sec. II), for the GPU full-build test:

* e4:    the positive-energy 4c eigenvalues (4992, ascending);
* probes: h @ V for a seeded complex block V (4992 x 2) and V itself;
* rows:  rows 0, 1000, 2495, 2496, 4991 of h;
* dlu_probes: the oracle's DLU Hamiltonian (Eqs. dlutrans, r2ctransatom)
  applied to the same V.

Run from the repository root:  python tests/golden/make_ag13_full_reference.py
(about 10 minutes and 12 GB on 8 cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import oracle.routes as ox  # noqa: E402
from x2c_inputs import C_LIGHT  # noqa: E402
from x2c_inputs.configs import ag13_molecule  # noqa: E402

ROWS = [0, 1000, 2495, 2496, 4991]


def probe_block(n, seed=20130318):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))


def main():
    t0 = time.time()
    mol = ag13_molecule(0)
    n = 2 * mol.Ntot
    print(f"molecule: Ntot {mol.Ntot}, coupling scale {mol.scale:.3e}", flush=True)
    h, eps = ox.x2c_direct(mol.S, mol.T, mol.V, mol.W, C_LIGHT, True)
    print(f"x2c_direct done ({time.time() - t0:.0f} s)", flush=True)
    e4 = oracle.dirac_positive_spectrum(mol.S, mol.T, mol.V, mol.W, C_LIGHT, True)
    print(f"4c spectrum done ({time.time() - t0:.0f} s)", flush=True)
    V = probe_block(n)
    hd = ox.x2c_dlu(mol.S, mol.T, mol.V, mol.W, mol.Ns, C_LIGHT, True)
    print(f"DLU done ({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ag13_full_seed0.npz")
    np.savez_compressed(out, e4=e4, eps=eps, V=V, probes=h @ V, rows=h[ROWS], row_index=np.array(ROWS),
                        dlu_probes=hd @ V, hmax=np.abs(h).max(), coupling_scale=mol.scale)
    print(f"wrote {out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
