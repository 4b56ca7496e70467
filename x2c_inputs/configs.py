"""Seeded synthetic workloads (stand-ins for the paper's Ag basis sets and
cluster geometries, which are not available).

Every workload is a list of one-centre atomic blocks built from even-tempered
uncontracted Gaussian shells with the closed-form integrals of
:mod:`x2c_inputs.integrals`.

* ``neon_s20``      : Z = 10, 20 s primitives alpha_k = 0.05 * 3^k, spin-free.
* ``ag_2c``         : Z = 47, s22 p18 d12 f8 (N = 192 scalar functions,
                      384 spinors), two-component.
* ``mixed_dlu``     : 512 blocks with Z drawn uniformly from
                      {1, 6, 8, 17, 29, 47, 79}; shell counts per Z below.
* ``ag309_dlu``     : 309 copies of the Z = 47 block with V and W scaled by a
                      per-atom factor U(0.98, 1.02) (equivalent to a slightly
                      perturbed nuclear charge, so physics checks still hold).
"""
from __future__ import annotations

import numpy as np

from .integrals import AtomBlock, Shell, build_block, even_tempered, scale_potential

# speed of light in atomic units used by the workloads (CODATA 2018)
C_LIGHT = 137.035999084
# the value quoted in the paper (Sec. IV)
C_LIGHT_PAPER = 137.0359895

Z_CHOICES = (1, 6, 8, 17, 29, 47, 79)

# even-tempered recipes per l: (alpha0, beta)
RECIPE = {0: (0.02, 2.6), 1: (0.03, 2.6), 2: (0.05, 2.7), 3: (0.2, 2.8)}


def shell_counts(Z: int) -> dict[int, int]:
    s = 10 + Z // 4
    p = 3 if Z < 3 else 4 + Z // 5
    d = max(1, Z // 6)
    f = Z // 10 if Z >= 29 else 0
    return {0: s, 1: p, 2: d, 3: f}


def shells_for(counts: dict[int, int]) -> list[Shell]:
    out = []
    for l in sorted(counts):
        if counts[l] > 0:
            a0, beta = RECIPE[l]
            out.append(Shell(l, even_tempered(a0, beta, counts[l])))
    return out


def neon_s20() -> AtomBlock:
    return build_block(10.0, [Shell(0, even_tempered(0.05, 3.0, 20))])


def ag_2c() -> AtomBlock:
    return build_block(47.0, shells_for({0: 22, 1: 18, 2: 12, 3: 8}))


def atom_block(Z: int) -> AtomBlock:
    return build_block(float(Z), shells_for(shell_counts(Z)))


def mixed_dlu(seed: int, nblocks: int = 512) -> list[AtomBlock]:
    rng = np.random.default_rng(seed)
    Zs = rng.choice(np.array(Z_CHOICES), size=nblocks)
    cache: dict[int, AtomBlock] = {}
    out = []
    for Z in Zs:
        Z = int(Z)
        if Z not in cache:
            cache[Z] = atom_block(Z)
        out.append(cache[Z])
    return out


def ag309_factors(seed: int, nblocks: int = 309) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.98, 1.02, size=nblocks)


def ag309_dlu(seed: int, nblocks: int = 309) -> list[AtomBlock]:
    base = ag_2c()
    return [scale_potential(base, float(f)) for f in ag309_factors(seed, nblocks)]


def pack_blocks(blocks: list[AtomBlock], twocomp: bool):
    """Pack blocks into flat float64 arrays in the library's batched layout.

    S, T, V: block b's N_b x N_b row-major matrix starts at in_off[b].
    W: spin-free -> W^0 at in_off[b]; two-component -> [W^0, W^x, W^y, W^z]
    contiguous at 4*in_off[b].
    Returns dict with S, T, V, W, Ns, in_off.
    """
    Ns = np.array([b.N for b in blocks], dtype=np.int32)
    sz = Ns.astype(np.int64) ** 2
    in_off = np.zeros(len(blocks), dtype=np.int64)
    if len(blocks) > 1:
        in_off[1:] = np.cumsum(sz)[:-1]
    total = int(sz.sum())
    S = np.empty(total)
    T = np.empty(total)
    V = np.empty(total)
    W = np.empty(total * (4 if twocomp else 1))
    for b, o, n2 in zip(blocks, in_off, sz):
        S[o:o + n2] = b.S.ravel()
        T[o:o + n2] = b.T.ravel()
        V[o:o + n2] = b.V.ravel()
        if twocomp:
            W[4 * o:4 * o + 4 * n2] = b.W.ravel()
        else:
            W[o:o + n2] = b.W[0].ravel()
    return dict(S=S, T=T, V=V, W=W, Ns=Ns, in_off=in_off)


# ----------------------------------------------------------------------------
# coupled molecules (full molecular matrices for the DLU assembly)
# ----------------------------------------------------------------------------

class Molecule:
    """Molecular scalar matrices over the atom-ordered basis: atom A's
    functions occupy scalar indices off[A] .. off[A] + Ns[A]."""

    def __init__(self, Z, S, T, V, W, Ns, scale):
        self.Z = list(Z)
        self.S, self.T, self.V, self.W = S, T, V, W      # W: (4, Ntot, Ntot)
        self.Ns = np.asarray(Ns, dtype=np.int32)
        self.off = np.concatenate([[0], np.cumsum(self.Ns)[:-1]]).astype(np.int64)
        self.scale = scale

    @property
    def Ntot(self) -> int:
        return int(self.Ns.sum())

    def atom(self, A: int) -> AtomBlock:
        o, n = int(self.off[A]), int(self.Ns[A])
        sl = slice(o, o + n)
        return AtomBlock(self.Z[A], self.S[sl, sl].copy(), self.T[sl, sl].copy(), self.V[sl, sl].copy(),
                         self.W[:, sl, sl].copy())


def coupled_molecule(blocks: list[AtomBlock], seed: int, scale: float = 1e-3) -> Molecule:
    """Block-diagonal molecular matrices from atomic blocks plus a seeded
    symmetric inter-atomic coupling: for scalar i, j on different atoms,
    M_ij += scale exp(-|i - j| / 50) u_ij sqrt(|M_ii M_jj|), u_ij = u_ji ~ U(-1, 1),
    for M in {S, T, V, W^0} (W^x, W^y, W^z stay atom-diagonal).  The scale is
    halved until the smallest eigenvalues of S and T are at least half of
    their block-diagonal values, so both stay positive definite."""
    Ns = [b.N for b in blocks]
    Ntot = int(sum(Ns))
    off = np.concatenate([[0], np.cumsum(Ns)[:-1]])
    S0 = np.zeros((Ntot, Ntot)); T0 = np.zeros((Ntot, Ntot)); V0 = np.zeros((Ntot, Ntot))
    W0 = np.zeros((4, Ntot, Ntot))
    atom_of = np.zeros(Ntot, dtype=np.int64)
    for A, (b, o) in enumerate(zip(blocks, off)):
        sl = slice(int(o), int(o) + b.N)
        S0[sl, sl] = b.S; T0[sl, sl] = b.T; V0[sl, sl] = b.V; W0[:, sl, sl] = b.W
        atom_of[sl] = A
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(Ntot, Ntot))
    u = np.triu(u, 1)
    u = u + u.T
    idx = np.arange(Ntot)
    shape = np.exp(-np.abs(idx[:, None] - idx[None, :]) / 50.0) * u
    shape[atom_of[:, None] == atom_of[None, :]] = 0.0
    lmin_s = np.linalg.eigvalsh(S0)[0]
    lmin_t = np.linalg.eigvalsh(T0)[0]

    def couple(M):
        d = np.sqrt(np.abs(np.diag(M)))
        return shape * np.outer(d, d)

    cS, cT, cV, cW = couple(S0), couple(T0), couple(V0), couple(W0[0])
    s = scale
    for _ in range(60):
        S = S0 + s * cS
        T = T0 + s * cT
        if np.linalg.eigvalsh(S)[0] >= 0.5 * lmin_s and np.linalg.eigvalsh(T)[0] >= 0.5 * lmin_t:
            break
        s *= 0.5
    V = V0 + s * cV
    W = W0.copy()
    W[0] = W0[0] + s * cW
    return Molecule([b.Z for b in blocks], S, T, V, W, Ns, s)


def ag13_molecule(seed: int = 0) -> Molecule:
    """Thirteen Z = 47 two-component blocks (4992 spinors) with the coupling
    above: the full-versus-DLU workload."""
    return coupled_molecule([ag_2c() for _ in range(13)], seed)
