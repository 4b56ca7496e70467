"""CPU FP64 oracle for the X2C one-electron Hamiltonian (test infrastructure).

This module is the reference that the GPU path is checked against.  It is
plain, slow NumPy/SciPy code in float64/complex128 and shares nothing with the
HIP library.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it.

Three independent routes compute the same matrix function h = H(S, T, V, W)
(Sec. II, Eq. r2ctrans):

* :func:`x2c_direct`   -- the non-orthogonal-basis route: generalized
  eigenproblem of the modified Dirac equation (Eq. moddiraceq), selection of
  the positive-energy branch (Sec. II, epsilon + c^2 > 0), X = C_S C_L^-1
  (Appendix, Eq. defxmat), renormalisation U^L = R =
  S^-1/2 (S^-1/2 S~ S^-1/2)^-1/2 S^1/2 with S~ = S + X^H T X / 2c^2 and
  U^S = X R (Eq. ulsnonortho), then h from Eq. utrans.
* :func:`x2c_kbasis`   -- the orthonormal kinetic-eigenbasis route of
  Sec. II.A: T K = S K t (Eq. orthonormalk), the transformed 4c matrix
  H^p built from V~ and W~, its standard Hermitian diagonalisation
  (Eq. diaghdp), X' (Eq. defxortho), R' = (I + X'^H X')^-1/2 (Eq. defrenorm)
  and the final back-transformed Hamiltonian.
* :func:`x2c_polar`    -- a Cholesky-reduced route: with S = L_S L_S^H and the
  reduced 4c matrix A = L_M^-1 D L_M^-H, orthonormal positive-energy
  eigenvectors Y = [Y_L; Y_S] of A give h = L_S U eps U^H L_S^H where
  Y_L = P U is the polar decomposition of the large-component block.  (This
  follows from the Appendix identities: the decoupled 2c eigenvectors are
  R^-1 C_L and they are S-orthonormal.)

The Appendix of the paper proves the first two routes equal; the third is
an algebraic consequence of the same definitions.  All three are
cross-checked in the tests.

Conventions: two-component matrices are in the spin-orbital basis
{lambda} x {alpha, beta} ordered [all alpha; all beta] (Eq. defstv), with W
assembled from W^0, W^x, W^y, W^z as in Eq. defw.  Spin-free mode drops
W^x, W^y, W^z and works with real N x N matrices (Sec. II, scalar
approximation).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------
# spinor-space assembly (Eqs. defstv and defw)
# ----------------------------------------------------------------------------

def spin_blockdiag(A: np.ndarray) -> np.ndarray:
    """diag(A, A) as a complex 2N x 2N matrix (Eq. defstv)."""
    N = A.shape[0]
    out = np.zeros((2 * N, 2 * N), dtype=complex)
    out[:N, :N] = A
    out[N:, N:] = A
    return out


def assemble_w(W0, Wx, Wy, Wz) -> np.ndarray:
    """W = [[W0 + i Wz, Wy + i Wx], [-Wy + i Wx, W0 - i Wz]] (Eq. defw)."""
    N = W0.shape[0]
    W = np.zeros((2 * N, 2 * N), dtype=complex)
    W[:N, :N] = W0 + 1j * Wz
    W[:N, N:] = Wy + 1j * Wx
    W[N:, :N] = -Wy + 1j * Wx
    W[N:, N:] = W0 - 1j * Wz
    return W


def spinor_matrices(S, T, V, W, twocomp: bool):
    """Return the (S, T, V, W) matrices of the chosen mode.

    W is either a single N x N W^0 (spin-free) or an array of shape
    (4, N, N) holding W^0, W^x, W^y, W^z.
    """
    W = np.asarray(W)
    if twocomp:
        return (spin_blockdiag(S), spin_blockdiag(T), spin_blockdiag(V),
                assemble_w(W[0], W[1], W[2], W[3]))
    W0 = W[0] if W.ndim == 3 else W
    return (np.array(S, dtype=float), np.array(T, dtype=float),
            np.array(V, dtype=float), np.array(W0, dtype=float))


def dirac_matrices(S, T, V, W, c: float):
    """D and M of the modified Dirac equation (Eq. moddiraceq):
    D = [[V, T], [T, W/4c^2 - T]],  M = diag(S, T/2c^2)."""
    n = S.shape[0]
    dt = np.result_type(S, T, V, W)
    D = np.zeros((2 * n, 2 * n), dtype=dt)
    M = np.zeros((2 * n, 2 * n), dtype=dt)
    D[:n, :n] = V
    D[:n, n:] = T
    D[n:, :n] = T
    D[n:, n:] = W / (4.0 * c * c) - T
    M[:n, :n] = S
    M[n:, n:] = T / (2.0 * c * c)
    return D, M


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

class X2CError(RuntimeError):
    pass


def herm_function(A: np.ndarray, f) -> np.ndarray:
    """f(A) for Hermitian A via its eigendecomposition A = C a C^H
    (Sec. III: A^-1/2 = C a^-1/2 C^H, principal branch)."""
    a, C = np.linalg.eigh(A)
    return (C * f(a)) @ C.conj().T


def positive_branch(e: np.ndarray, C: np.ndarray, c: float, n: int):
    """Keep the eigenpairs with epsilon + c^2 > 0 (Sec. II)."""
    keep = e + c * c > 0.0
    if int(keep.sum()) != n:
        raise X2CError(f"positive-energy count {int(keep.sum())} != {n}")
    return e[keep], C[:, keep]


def dirac_positive_spectrum(S, T, V, W, c: float, twocomp: bool) -> np.ndarray:
    """Positive-energy eigenvalues of the 4c modified Dirac equation,
    ascending (brute force: generalized eigensolve of (D, M))."""
    Sx, Tx, Vx, Wx = spinor_matrices(S, T, V, W, twocomp)
    D, M = dirac_matrices(Sx, Tx, Vx, Wx, c)
    e = sla.eigh(D, M, eigvals_only=True)
    n = Sx.shape[0]
    e = e[e + c * c > 0.0]
    if e.size != n:
        raise X2CError(f"positive-energy count {e.size} != {n}")
    return e


def spectrum_of(h: np.ndarray, S, twocomp: bool) -> np.ndarray:
    """Eigenvalues of the 2c (or 1c) electrons-only equation h C = S C eps
    (Eq. 2ceoeq), ascending.  Used to score any computed h."""
    Sx = spin_blockdiag(S) if twocomp else np.asarray(S, dtype=float)
    hh = 0.5 * (h + h.conj().T)
    return sla.eigh(hh, Sx, eigvals_only=True)


# ----------------------------------------------------------------------------
# route 1: non-orthogonal basis (Eqs. moddiraceq, defxmat, ulsnonortho, utrans)
# ----------------------------------------------------------------------------

def x2c_direct(S, T, V, W, c: float, twocomp: bool, return_parts: bool = False):
    """h and the positive-energy spectrum by the literal definition.

    Steps, in the paper's notation:
      1. D C = M C eps (Eq. moddiraceq), generalized Hermitian eigensolve.
      2. keep epsilon + c^2 > 0; C_L, C_S = upper and lower halves.
      3. X = C_S C_L^-1 (Eq. defxmat).
      4. S~ = S + X^H T X / 2c^2;  R = S^-1/2 (S^-1/2 S~ S^-1/2)^-1/2 S^1/2
         (Eq. ulnonortho);  U^L = R,  U^S = X R (Eq. usnonortho).
      5. h = [U^L^H  U^S^H] D [U^L; U^S] (Eq. utrans)
           = R^H (V + T X + X^H T + X^H (W/4c^2 - T) X) R.
    """
    Sx, Tx, Vx, Wx = spinor_matrices(S, T, V, W, twocomp)
    n = Sx.shape[0]
    D, M = dirac_matrices(Sx, Tx, Vx, Wx, c)
    e, C = sla.eigh(D, M)
    eps, Cp = positive_branch(e, C, c, n)
    CL = Cp[:n]
    CS = Cp[n:]
    # X C_L = C_S  ->  C_L^T X^T = C_S^T
    X = np.linalg.solve(CL.T, CS.T).T
    St = Sx + X.conj().T @ Tx @ X / (2.0 * c * c)
    S_mh = herm_function(Sx, lambda s: s ** -0.5)
    S_h = herm_function(Sx, lambda s: s ** 0.5)
    Q = S_mh @ St @ S_mh
    Q_mh = herm_function(Q, lambda q: q ** -0.5)
    R = S_mh @ Q_mh @ S_h
    UL = R
    US = X @ R
    Wp = Wx / (4.0 * c * c) - Tx
    h = (UL.conj().T @ Vx @ UL + UL.conj().T @ Tx @ US
         + US.conj().T @ Tx @ UL + US.conj().T @ Wp @ US)
    if return_parts:
        L = Vx + Tx @ X + X.conj().T @ Tx + X.conj().T @ Wp @ X
        return h, eps, dict(X=X, St=St, R=R, L=L, Q=Q)
    return h, eps


# ----------------------------------------------------------------------------
# picture change of property operators (Sec. II: U^L and U^S are kept for the
# picture-change transformation of property integrals; Eq. utrans)
# ----------------------------------------------------------------------------

def property_blocks(O, WO, c: float, twocomp: bool):
    """4c matrix of a multiplicative one-electron operator O in the basis of
    the modified Dirac equation (Eq. moddiraceq: large components chi, small
    components sigma.p chi / 2c): P_LL = O (spin-diagonal, Eq. defstv),
    P_LS = P_SL = 0, P_SS = W^O / 4c^2 with W^O = <sigma.p chi|O|sigma.p chi>
    in the form of Eq. defw.  WO: (4, N, N) for two-component, W^O0 (N x N)
    or (4, N, N) for spin-free."""
    WO = np.asarray(WO)
    if twocomp:
        PLL = spin_blockdiag(O)
        PSS = assemble_w(WO[0], WO[1], WO[2], WO[3]) / (4.0 * c * c)
    else:
        PLL = np.array(O, dtype=float)
        PSS = np.array(WO[0] if WO.ndim == 3 else WO, dtype=float) / (4.0 * c * c)
    zero = np.zeros_like(PLL)
    return PLL, zero, zero.copy(), PSS


def picture_change(PLL, PLS, PSL, PSS, X, R):
    """Eq. utrans with a property's 4c matrix P = [[P_LL, P_LS], [P_SL, P_SS]]
    in place of D, and the decoupling U^L = R, U^S = X R (Eqs. ulnonortho,
    usnonortho): [U^L^H U^S^H] P [U^L; U^S]."""
    UL = R
    US = X @ R
    return (UL.conj().T @ PLL @ UL + UL.conj().T @ PLS @ US
            + US.conj().T @ PSL @ UL + US.conj().T @ PSS @ US)


# ----------------------------------------------------------------------------
# route 2: orthonormal kinetic eigenbasis (Sec. II.A)
# ----------------------------------------------------------------------------

def x2c_kbasis(S, T, V, W, c: float, twocomp: bool):
    """h by the paper's own route (Eqs. orthonormalk, propk, defk, diaghdp,
    defxortho, defrenorm and the final back transformation)."""
    S = np.asarray(S, dtype=float)
    T = np.asarray(T, dtype=float)
    V = np.asarray(V, dtype=float)
    W = np.asarray(W, dtype=float)
    N = S.shape[0]
    # T K = S K t  with  K^T S K = I, K^T T K = t  (Eq. orthonormalk, propk)
    t, K = sla.eigh(T, S)
    if np.any(t <= 0.0):
        raise X2CError("kinetic matrix not positive definite")
    p = np.sqrt(2.0 * t)                       # momentum eigenvalues
    Kinv = np.linalg.inv(K)
    Vt = K.T @ V @ K                           # V~ = K^T V K (scalar level)
    Wq = W if W.ndim == 3 else W[None]
    Wt_q = [(K.T @ Wk @ K) / np.outer(p, p) for Wk in (Wq if twocomp else Wq[:1])]
    if twocomp:
        Vt2 = spin_blockdiag(Vt)
        Wt = assemble_w(*Wt_q)
        p2 = np.concatenate([p, p])
        Kinv2 = spin_blockdiag(Kinv)
    else:
        Vt2 = Vt
        Wt = Wt_q[0]
        p2 = p
        Kinv2 = Kinv
    n = Vt2.shape[0]
    cp = np.diag(c * p2)
    Hp = np.zeros((2 * n, 2 * n), dtype=np.result_type(Vt2, Wt))
    Hp[:n, :n] = Vt2
    Hp[:n, n:] = cp
    Hp[n:, :n] = cp
    Hp[n:, n:] = Wt - 2.0 * c * c * np.eye(n)
    e, C = np.linalg.eigh(Hp)                  # Eq. diaghdp
    eps, Cp = positive_branch(e, C, c, n)
    CLp = Cp[:n]
    CSp = Cp[n:]
    Xp = np.linalg.solve(CLp.T, CSp.T).T       # X' = C_S' C_L'^-1 (Eq. defxortho)
    Rp = herm_function(np.eye(n) + Xp.conj().T @ Xp, lambda q: q ** -0.5)  # Eq. defrenorm
    inner = (Vt2 + (c * p2)[:, None] * Xp + Xp.conj().T * (c * p2)[None, :]
             + Xp.conj().T @ (Wt - 2.0 * c * c * np.eye(n)) @ Xp)
    B = Rp @ Kinv2
    h = B.conj().T @ inner @ B
    return h, eps


# ----------------------------------------------------------------------------
# route 3: Cholesky reduction + polar decomposition
# ----------------------------------------------------------------------------

def reduced_dirac(S, T, V, W, c: float, twocomp: bool):
    """Cholesky-reduced 4c matrix A = L_M^-1 D L_M^-H with
    M = L_M L_M^H, L_M = diag(L_S, L_T / (sqrt(2) c)).  Returns (A, L_S, L_T)
    in spinor space."""
    Sx, Tx, Vx, Wx = spinor_matrices(S, T, V, W, twocomp)
    LS = np.linalg.cholesky(Sx)
    LT = np.linalg.cholesky(Tx)
    D, _ = dirac_matrices(Sx, Tx, Vx, Wx, c)
    n = Sx.shape[0]
    LM = np.zeros((2 * n, 2 * n), dtype=LS.dtype)
    LM[:n, :n] = LS
    LM[n:, n:] = LT / (np.sqrt(2.0) * c)
    Y = sla.solve_triangular(LM, D, lower=True)
    A = sla.solve_triangular(LM, Y.conj().T, lower=True).conj().T
    return A, LS, LT


def x2c_polar(S, T, V, W, c: float, twocomp: bool):
    """h = L_S U eps U^H L_S^H, with Y_L = P U (polar) from the orthonormal
    positive-energy eigenvectors of the reduced matrix."""
    A, LS, _ = reduced_dirac(S, T, V, W, c, twocomp)
    n = LS.shape[0]
    e, Y = np.linalg.eigh(A)
    eps, Yp = positive_branch(e, Y, c, n)
    YL = Yp[:n]
    Wl, _, Vh = np.linalg.svd(YL)
    U = Wl @ Vh
    G = LS @ U
    h = (G * eps[None, :]) @ G.conj().T
    return h, eps


def x2c(S, T, V, W, c: float, twocomp: bool):
    """Default oracle entry point (route 1)."""
    return x2c_direct(S, T, V, W, c, twocomp)


# ----------------------------------------------------------------------------
# DLU molecular Hamiltonian (Sec. III.A)
# ----------------------------------------------------------------------------

def atom_spinor_index(off: int, N: int, Ntot: int, twocomp: bool) -> np.ndarray:
    """Molecular spin-orbital indices of an atom's functions in its own
    [alpha; beta] order (molecular order: all alpha, then all beta)."""
    a = np.arange(off, off + N)
    return np.concatenate([a, Ntot + a]) if twocomp else a


def x2c_dlu(S, T, V, W, Ns, c: float, twocomp: bool, return_parts: bool = False):
    """Molecular h in the diagonal local approximation to the unitary
    transformation: U^L and U^S are direct sums of atomic blocks (Eq.
    dlutrans), each evaluated from the atom's own diagonal blocks of S, T, V, W
    (Eq. r2ctransatom), and h follows from Eq. utrans with the full molecular
    matrices:  h = U^L^H V U^L + U^L^H T U^S + U^S^H T U^L + U^S^H (W/4c^2 - T) U^S.

    S, T, V: Ntot x Ntot; W: (4, Ntot, Ntot) (two-component) or W^0."""
    Ns = [int(x) for x in Ns]
    Ntot = int(sum(Ns))
    W = np.asarray(W)
    Sx, Tx, Vx, Wx = spinor_matrices(S, T, V, W, twocomp)
    n = Sx.shape[0]
    UL = np.zeros((n, n), dtype=Sx.dtype)
    US = np.zeros((n, n), dtype=Sx.dtype)
    parts = []
    off = 0
    for NA in Ns:
        sl = slice(off, off + NA)
        WA = W[:, sl, sl] if W.ndim == 3 else W[sl, sl]
        if not twocomp and W.ndim == 3:
            WA = WA[0]
        _, _, p = x2c_direct(S[sl, sl], T[sl, sl], V[sl, sl], WA, c, twocomp, return_parts=True)
        idx = atom_spinor_index(off, NA, Ntot, twocomp)
        UL[np.ix_(idx, idx)] = p["R"]
        US[np.ix_(idx, idx)] = p["X"] @ p["R"]
        parts.append(dict(X=p["X"], R=p["R"]))
        off += NA
    Wp = Wx / (4.0 * c * c) - Tx
    h = (UL.conj().T @ Vx @ UL + UL.conj().T @ Tx @ US
         + US.conj().T @ Tx @ UL + US.conj().T @ Wp @ US)
    if return_parts:
        return h, parts
    return h


def x2c_dlu_pair(T, V, W, Ns, A: int, B: int, parts, c: float, twocomp: bool):
    """One atom-pair block h_AB of the DLU Hamiltonian, i.e. Eq. utrans
    restricted to the rows of atom A and the columns of atom B with the
    block-diagonal U of Eq. dlutrans:
    h_AB = U^L_AA^H V_AB U^L_BB + U^L_AA^H T_AB U^S_BB + U^S_AA^H T_AB U^L_BB
           + U^S_AA^H (W_AB/4c^2 - T_AB) U^S_BB,
    with parts[A] = dict(X=X_A, R=R_A) (U^L_AA = R_A, U^S_AA = X_A R_A)."""
    Ns = [int(x) for x in Ns]
    Ntot = int(sum(Ns))
    off = np.concatenate([[0], np.cumsum(Ns)[:-1]]).astype(int)
    W = np.asarray(W)
    Tx, Vx, Wx = spinor_matrices(T, T, V, W, twocomp)[1:]
    ia = atom_spinor_index(off[A], Ns[A], Ntot, twocomp)
    ib = atom_spinor_index(off[B], Ns[B], Ntot, twocomp)
    sub = lambda M: M[np.ix_(ia, ib)]
    ULa, ULb = parts[A]["R"], parts[B]["R"]
    USa, USb = parts[A]["X"] @ ULa, parts[B]["X"] @ ULb
    Wp = sub(Wx) / (4.0 * c * c) - sub(Tx)
    return (ULa.conj().T @ sub(Vx) @ ULb + ULa.conj().T @ sub(Tx) @ USb
            + USa.conj().T @ sub(Tx) @ ULb + USa.conj().T @ Wp @ USb)
