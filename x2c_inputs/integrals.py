"""Closed-form one-centre integrals over uncontracted spherical Gaussians.

This module only *generates inputs*: the four real matrices S, T, V, W^0 and
the spin-orbit matrices W^x, W^y, W^z that the relativistic transformation
consumes (Sec. II, Eqs. defstv, defw and the W^q subequations).  It holds none
of the decoupling arithmetic and is shared by the CPU oracle, the tests and the
benchmark driver.

Primitive functions are  chi(r) = r^l exp(-a r^2) S_lm(r_hat)  with real
spherical harmonics normalised on the unit sphere.  All functions sit on one
centre (a DLU atomic block, Sec. III.A, Eq. r2ctransatom) with a point nucleus
of charge Z (Sec. IV), so every scalar integral is diagonal in (l, m).  With
p = a + b the radial integrals are

    S   = Gamma(l + 3/2) / (2 p^(l+3/2))
    T   = (2l + 3) (a b / p) S                       (T = <grad chi_a . grad chi_b>/2)
    V   = -Z l! / (2 p^(l+1))                        (V = -Z / r)
    W^0 = -Z [ [l>=1] l!/(2 p^l) + 2 a b (l+1)!/p^(l+2) ]   (<grad chi_a . V grad chi_b>)
    W^k = -Z (l-1)!/(2 p^l) * A^k_{m m'}             (k = x, y, z; l >= 1)

where A^k = <S_lm | (r x grad)_k | S_lm'> is real antisymmetric.  The W^k form
follows from the definition W^k_ij = <p_i V p_j - p_j V p_i> of Eq. defw by
integration by parts: W^k_ij = int V (grad chi_i x grad chi_j)_k, and for a
central potential -Z/r this is -Z <chi_i| r^-3 (r x grad)_k |chi_j>.

Basis order inside a block: shells by l ascending (s, p, d, f), then exponent
index ascending, then m = -l .. l.  The generator returns matrices over
*normalised* primitives (S_ii = 1); spectra are unchanged by this diagonal
congruence.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------
# real spherical harmonics: angular momentum matrices
# ----------------------------------------------------------------------------

def complex_to_real_harmonics(l: int) -> np.ndarray:
    """Rows give the real harmonic S_{l,m} (m = -l..l) as a combination of
    the complex Y_{l,m'} (m' = -l..l, Condon-Shortley phase):

        S_{l,0}    = Y_{l,0}
        S_{l,m>0}  = [(-1)^m Y_{l,m} + Y_{l,-m}] / sqrt 2
        S_{l,-m}   = i [Y_{l,-m} - (-1)^m Y_{l,m}] / sqrt 2    (m > 0)

    With this choice S_{1,1} ~ x, S_{1,-1} ~ y, S_{1,0} ~ z.
    """
    dim = 2 * l + 1
    U = np.zeros((dim, dim), dtype=complex)
    s2 = 1.0 / math.sqrt(2.0)
    for m in range(-l, l + 1):
        row = m + l
        if m == 0:
            U[row, l] = 1.0
        elif m > 0:
            U[row, m + l] = (-1) ** m * s2
            U[row, -m + l] = s2
        else:
            am = -m
            U[row, -am + l] = 1j * s2
            U[row, am + l] = -1j * (-1) ** am * s2
    return U


def rxgrad_real(l: int) -> np.ndarray:
    """A^k_{m m'} = <S_lm | (r x grad)_k | S_lm'> for k = x, y, z.

    Built from the ladder-operator form of L in the complex basis
    (L_z |m> = m |m>, L_+ |m> = sqrt(l(l+1) - m(m+1)) |m+1>) and the
    identity r x grad = i L.  Returns a real array of shape (3, 2l+1, 2l+1);
    each A^k is antisymmetric.
    """
    dim = 2 * l + 1
    ms = np.arange(-l, l + 1)
    Lz = np.diag(ms).astype(complex)
    Lp = np.zeros((dim, dim), dtype=complex)
    for m in range(-l, l):
        Lp[m + 1 + l, m + l] = math.sqrt(l * (l + 1) - m * (m + 1))
    Lm = Lp.conj().T
    Lx = 0.5 * (Lp + Lm)
    Ly = -0.5j * (Lp - Lm)
    U = complex_to_real_harmonics(l)
    out = np.zeros((3, dim, dim))
    for k, Lk in enumerate((Lx, Ly, Lz)):
        Lreal = U.conj() @ Lk @ U.T          # <S_a|L_k|S_b>
        Ak = 1j * Lreal
        if np.abs(Ak.imag).max() > 1e-13:
            raise AssertionError("r x grad is not real in the real-harmonic basis")
        out[k] = Ak.real
    out[np.abs(out) < 1e-15] = 0.0
    return out


# ----------------------------------------------------------------------------
# radial closed forms
# ----------------------------------------------------------------------------

def radial_S(l: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    p = a + b
    return math.gamma(l + 1.5) / (2.0 * p ** (l + 1.5))


def radial_T(l: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    p = a + b
    return (2 * l + 3) * a * b / p * radial_S(l, a, b)


def radial_V(l: int, a: np.ndarray, b: np.ndarray, Z: float) -> np.ndarray:
    p = a + b
    return -Z * math.factorial(l) / (2.0 * p ** (l + 1))


def radial_W0(l: int, a: np.ndarray, b: np.ndarray, Z: float) -> np.ndarray:
    p = a + b
    t = 2.0 * a * b * math.factorial(l + 1) / p ** (l + 2)
    if l >= 1:
        t = t + math.factorial(l) / (2.0 * p ** l)
    return -Z * t


def radial_Wso(l: int, a: np.ndarray, b: np.ndarray, Z: float) -> np.ndarray:
    """Radial factor of W^k: -Z int r^(2l-1) exp(-p r^2) dr (l >= 1)."""
    p = a + b
    return -Z * math.factorial(l - 1) / (2.0 * p ** l)


# ----------------------------------------------------------------------------
# blocks
# ----------------------------------------------------------------------------

@dataclass
class Shell:
    l: int
    exponents: np.ndarray   # ascending


@dataclass
class AtomBlock:
    """Integrals of one DLU atomic block (Sec. III.A, Eq. r2ctransatom)."""
    Z: float
    S: np.ndarray            # (N, N)
    T: np.ndarray
    V: np.ndarray
    W: np.ndarray            # (4, N, N): W^0, W^x, W^y, W^z

    @property
    def N(self) -> int:
        return self.S.shape[0]


def even_tempered(alpha0: float, beta: float, count: int) -> np.ndarray:
    return alpha0 * beta ** np.arange(count, dtype=float)


def build_block(Z: float, shells: list[Shell], normalise: bool = True) -> AtomBlock:
    """Assemble S, T, V, W^0..z for one centre from its shells."""
    # index bookkeeping
    sizes = [len(sh.exponents) * (2 * sh.l + 1) for sh in shells]
    N = int(sum(sizes))
    S = np.zeros((N, N))
    T = np.zeros((N, N))
    V = np.zeros((N, N))
    W = np.zeros((4, N, N))
    off = 0
    for sh, size in zip(shells, sizes):
        l = sh.l
        nexp = len(sh.exponents)
        dim = 2 * l + 1
        a = sh.exponents[:, None]
        b = sh.exponents[None, :]
        rs = radial_S(l, a, b)
        rt = radial_T(l, a, b)
        rv = radial_V(l, a, b, Z)
        rw = radial_W0(l, a, b, Z)
        Ak = rxgrad_real(l) if l >= 1 else None
        rso = radial_Wso(l, a, b, Z) if l >= 1 else None
        # function index = off + k*dim + (m + l)
        for i in range(nexp):
            for j in range(nexp):
                bi = off + i * dim
                bj = off + j * dim
                for mm in range(dim):
                    S[bi + mm, bj + mm] = rs[i, j]
                    T[bi + mm, bj + mm] = rt[i, j]
                    V[bi + mm, bj + mm] = rv[i, j]
                    W[0, bi + mm, bj + mm] = rw[i, j]
                if l >= 1:
                    for k in range(3):
                        W[1 + k, bi:bi + dim, bj:bj + dim] = rso[i, j] * Ak[k]
        off += size
    if normalise:
        d = 1.0 / np.sqrt(np.diag(S))
        Dm = np.outer(d, d)
        S = S * Dm
        T = T * Dm
        V = V * Dm
        W = W * Dm[None]
        np.fill_diagonal(S, 1.0)
    return AtomBlock(Z=float(Z), S=S, T=T, V=V, W=W)


def s_only_block_unnormalised(Z: float, exponents: np.ndarray) -> AtomBlock:
    """Unnormalised s primitives exp(-a r^2): the four closed forms
    S = (pi/p)^1.5, T = 3ab/p S, V = -2 pi Z/p, W = -8 pi Z a b / p^2
    (the radial forms above times 4 pi).  Used to check the generator."""
    a = exponents[:, None]
    b = exponents[None, :]
    p = a + b
    S = (np.pi / p) ** 1.5
    T = 3.0 * a * b / p * S
    V = -2.0 * np.pi * Z / p
    W0 = -8.0 * np.pi * Z * a * b / p ** 2
    N = len(exponents)
    W = np.zeros((4, N, N))
    W[0] = W0
    return AtomBlock(Z=float(Z), S=S, T=T, V=V, W=W)


def scale_potential(blk: AtomBlock, f: float) -> AtomBlock:
    """Multiply V and all W^q by f (equivalent to nuclear charge f*Z)."""
    return AtomBlock(Z=blk.Z * f, S=blk.S.copy(), T=blk.T.copy(),
                     V=blk.V * f, W=blk.W * f)
