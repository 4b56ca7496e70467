"""CPU FP64 oracle for the X2C, BSS and DKHn Hamiltonians -- test
infrastructure only.

Imported by the tests, the smoke check and the benchmark's CPU-baseline leg;
never by the GPU library or its Python binding.
"""
from .routes import (X2CError, assemble_w, dirac_matrices, dirac_positive_spectrum,  # noqa: F401
                  atom_spinor_index, reduced_dirac, spectrum_of, spin_blockdiag, spinor_matrices,
                  x2c, x2c_direct, x2c_dlu, x2c_dlu_pair, x2c_kbasis, x2c_polar)
from .fw import bss, dkh, fpfw_blocks, kinetic_basis  # noqa: F401,E402
