"""Seeded synthetic inputs (closed-form one-centre Gaussian integrals).

Shared by the CPU oracle, the tests and the benchmark; contains no part of the
relativistic decoupling itself."""
from .integrals import AtomBlock, Shell, build_block, rxgrad_real  # noqa: F401
from .configs import (C_LIGHT, C_LIGHT_PAPER, Molecule, ag13_molecule, ag_2c, ag309_dlu,  # noqa: F401
                      atom_block, coupled_molecule, mixed_dlu, neon_s20, pack_blocks, shell_counts)
