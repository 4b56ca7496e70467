"""CPU FP64 oracle for the BSS and DKHn one-electron Hamiltonians (test
infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU legs, never by the GPU library or its binding).

Both methods start from the free-particle Foldy-Wouthuysen (fpFW)
transformation of the 4c matrix in the orthonormal kinetic basis (Sec. II):

* T K = S K t, K^T S K = I (Eq. orthonormalk, propk), p = sqrt(2 t);
* H^p = [[V~, c p], [c p, W~ - 2c^2]] with V~ = K^T V K and
  W~ = p^-1 K^T W K p^-1 (Sec. II.A);
* E_0 = sqrt(c^2 p^2 + c^4), U_0^A = sqrt((E_0 + c^2) / 2E_0),
  U_0^B = sqrt((E_0 - c^2) / 2E_0) (Sec. II, BSS approach);
* H^0 = [[E_1 + E_0 - c^2, O_1], [O_1^H, E_1' - E_0 - c^2]] with
  E_1  = U_0^A V~ U_0^A + U_0^B W~ U_0^B,
  O_1  = U_0^A V~ U_0^B - U_0^B W~ U_0^A,
  E_1' = U_0^B V~ U_0^B + U_0^A W~ U_0^A      (the block formula of H^0).

Reading (recorded in the design notes): the printed 4 x 4 form of the fpFW
matrix and the printed H^0 blocks differ by the sign of the negative-energy
basis vectors.  The H^0 blocks above follow when the transformation's
columns are [U_0^A; U_0^B] (the free particle's positive-energy solution in
the H^p basis) and [U_0^B; -U_0^A]; with that choice a positive-energy
vector [I; X''] of H^0 is [U_0^A + U_0^B X''; U_0^B - U_0^A X''] in the H^p
basis, so U^S_BSS carries (U_0^B - U_0^A X'') where the printed formula has
(U_0^A X'' - U_0^B).  Only this sign gives exact decoupling (pinned by the
renormalisation condition and by the spectrum in the tests).

E_0 - c^2 is evaluated as c^2 p^2 / (E_0 + c^2) (the same number without
the cancellation for small p).
"""
from __future__ import annotations

from math import factorial

import numpy as np
import scipy.linalg as sla

from .routes import X2CError, assemble_w, herm_function, positive_branch, spin_blockdiag


# ----------------------------------------------------------------------------
# orthonormal kinetic basis and the free-particle FW transformation
# ----------------------------------------------------------------------------

def kinetic_basis(S, T):
    """T K = S K t with K^T S K = I (Eqs. orthonormalk, propk); p = sqrt(2t)."""
    t, K = sla.eigh(np.asarray(T, dtype=float), np.asarray(S, dtype=float))
    if np.any(t <= 0.0):
        raise X2CError("kinetic matrix not positive definite")
    return K, t, np.sqrt(2.0 * t)


def free_particle(p, c: float):
    """E_0, E_0 - c^2, U_0^A, U_0^B on the momentum eigenvalues p."""
    E0 = np.sqrt(c * c * p * p + c ** 4)
    E0m = c * c * p * p / (E0 + c * c)              # E_0 - c^2
    UA = np.sqrt((E0 + c * c) / (2.0 * E0))
    UB = np.sqrt(E0m / (2.0 * E0))
    return E0, E0m, UA, UB


def fpfw_blocks(S, T, V, W, c: float, twocomp: bool):
    """Everything both methods need: K, p, E_0, U_0^A, U_0^B (spinor-space
    vectors), V~, W~ and the blocks E_1, O_1, E_1' of H^0.

    W is W^0 (spin-free, N x N or (4, N, N)) or (4, N, N) W^0, W^x, W^y, W^z;
    two-component W~ is assembled from the four W~^q as in Eq. defw."""
    K, t, p = kinetic_basis(S, T)
    V = np.asarray(V, dtype=float)
    W = np.asarray(W, dtype=float)
    Vt = K.T @ V @ K
    pinv = 1.0 / p
    if twocomp:
        Wq = [pinv[:, None] * (K.T @ W[q] @ K) * pinv[None, :] for q in range(4)]
        Vt = spin_blockdiag(Vt)
        Wt = assemble_w(*Wq)
        p2 = np.concatenate([p, p])
        Kx = spin_blockdiag(K)
    else:
        W0 = W[0] if W.ndim == 3 else W
        Wt = pinv[:, None] * (K.T @ W0 @ K) * pinv[None, :]
        p2 = p
        Kx = K
    E0, E0m, UA, UB = free_particle(p2, c)
    DA, DB = np.diag(UA), np.diag(UB)
    E1 = DA @ Vt @ DA + DB @ Wt @ DB
    O1 = DA @ Vt @ DB - DB @ Wt @ DA
    E1p = DB @ Vt @ DB + DA @ Wt @ DA
    return dict(K=Kx, p=p2, E0=E0, E0m=E0m, UA=UA, UB=UB, Vt=Vt, Wt=Wt, E1=E1, O1=O1, E1p=E1p)


def back_transform(hp, K):
    """The electronic matrix in the orthonormal basis back to the original
    basis: (K^-1)^H hp K^-1 (Sec. II.A)."""
    Kinv = np.linalg.inv(K)
    return Kinv.conj().T @ hp @ Kinv


# ----------------------------------------------------------------------------
# BSS (Sec. II, "The BSS approach", Eq. u1trafo)
# ----------------------------------------------------------------------------

def bss(S, T, V, W, c: float, twocomp: bool, return_parts: bool = False):
    """h_BSS in the paper's order: H^0, its standard Hermitian
    diagonalisation (positive-energy branch eps + c^2 > 0), X'' = C_S''
    C_L''^-1, R'' = (I + X''^H X'')^-1/2, U^L_BSS and U^S_BSS (with the sign
    reading of the module docstring), and h from Eq. utrans."""
    f = fpfw_blocks(S, T, V, W, c, twocomp)
    n = f["E1"].shape[0]
    c2 = c * c
    H0 = np.zeros((2 * n, 2 * n), dtype=np.result_type(f["E1"], f["O1"]))
    H0[:n, :n] = f["E1"] + np.diag(f["E0m"])
    H0[:n, n:] = f["O1"]
    H0[n:, :n] = f["O1"].conj().T
    H0[n:, n:] = f["E1p"] - np.diag(f["E0"] + c2)
    e, C = np.linalg.eigh(H0)
    eps, Cp = positive_branch(e, C, c, n)
    X2 = np.linalg.solve(Cp[:n].T, Cp[n:].T).T                 # X'' = C_S'' C_L''^-1
    R2 = herm_function(np.eye(n) + X2.conj().T @ X2, lambda q: q ** -0.5)
    K = f["K"]
    Kinv = np.linalg.inv(K)
    DA, DB = np.diag(f["UA"]), np.diag(f["UB"])
    UL = K @ (DA + DB @ X2) @ R2 @ Kinv
    US = 2.0 * c * K @ np.diag(1.0 / f["p"]) @ (DB - DA @ X2) @ R2 @ Kinv
    Sx, Tx, Vx, Wx = _spinor(S, T, V, W, twocomp)
    Wp = Wx / (4.0 * c2) - Tx
    h = (UL.conj().T @ Vx @ UL + UL.conj().T @ Tx @ US + US.conj().T @ Tx @ UL + US.conj().T @ Wp @ US)
    if return_parts:
        return h, eps, dict(UL=UL, US=US, X2=X2, R2=R2, H0=H0, **f)
    return h, eps


def _spinor(S, T, V, W, twocomp):
    from .routes import spinor_matrices
    return spinor_matrices(S, T, V, W, twocomp)


# ----------------------------------------------------------------------------
# DKHn with the exponential parametrisation (Sec. II, "The DKH approach")
# ----------------------------------------------------------------------------

def dkh(S, T, V, W, c: float, twocomp: bool, order: int, return_parts: bool = False):
    """h_DKHn: the fpFW Hamiltonian H^0 = D_0 + H_1 (D_0 = diag(E_0 - c^2,
    -E_0 - c^2), H_1 first order in the potential) is transformed by
    U_k = exp(W_k), k = 1, 2, ..., with the anti-Hermitian odd
    W_k = [[0, W_k], [-W_k^H, 0]] chosen so that the odd term of order k
    vanishes: [W_k, D_0] = -O_k, i.e. (W_k)_ij = (O_k)_ij / (E_0i + E_0j).
    Each step applies H -> exp(W) H exp(-W) = sum_i ad_W^i(H) / i! term by
    term, keeping every term of order <= n in the potential (a term of
    order l picks up k per commutator).  h_DKHn is the upper-left block of
    the even terms through order n, back-transformed by K^-1.

    The algorithm is the definition: full 4c block matrices, every
    commutator formed explicitly, no skipped products."""
    n_ord = int(order)
    if n_ord < 1:
        raise ValueError("order >= 1")
    f = fpfw_blocks(S, T, V, W, c, twocomp)
    n = f["E1"].shape[0]
    c2 = c * c
    dt = np.result_type(f["E1"], f["O1"])
    D0 = np.zeros((2 * n, 2 * n), dtype=dt)
    D0[:n, :n] = np.diag(f["E0m"])
    D0[n:, n:] = -np.diag(f["E0"] + c2)
    H1 = np.zeros((2 * n, 2 * n), dtype=dt)
    H1[:n, :n] = f["E1"]
    H1[:n, n:] = f["O1"]
    H1[n:, :n] = f["O1"].conj().T
    H1[n:, n:] = f["E1p"]
    terms = {0: D0, 1: H1}                       # order -> 4c matrix of that order
    denom = f["E0"][:, None] + f["E0"][None, :]
    Ws = []
    for k in range(1, n_ord + 1):
        Ok = terms.get(k, np.zeros_like(D0))[:n, n:]
        Wk = Ok / denom
        Wf = np.zeros_like(D0)
        Wf[:n, n:] = Wk
        Wf[n:, :n] = -Wk.conj().T
        Ws.append(Wk)
        new = {j: np.zeros_like(D0) for j in range(n_ord + 1)}
        for l, M in terms.items():
            A = M
            i = 0
            while l + i * k <= n_ord:
                new[l + i * k] += A / factorial(i)
                A = Wf @ A - A @ Wf
                i += 1
        terms = new
    hp = sum(terms[j][:n, :n] for j in range(n_ord + 1))
    h = back_transform(hp, f["K"])
    if return_parts:
        return h, dict(terms=terms, W=Ws, **f)
    return h


def dkh2_explicit(f):
    """E_2 = (W_1 O_1^H + c.t.) / 2 with W_1 = O_1 / (E_0i + E_0j) (the
    paper's DKH2 formula)."""
    W1 = f["O1"] / (f["E0"][:, None] + f["E0"][None, :])
    A = W1 @ f["O1"].conj().T
    return 0.5 * (A + A.conj().T)


def dkh3_explicit(f):
    """E_3 = (W_1 (W_1 E_1' - E_1 W_1)^H + c.t.) / 2: the odd second-order term
    [W_1, E_1] has the upper-right block W_1 E_1' - E_1 W_1 (the paper's
    commutator of W with an even matrix), and E_3 is half its commutator
    with W_1.  (The printed E_3 has E_1 and E_1' interchanged inside the
    bracket; this form is the one that follows from the commutators.)"""
    W1 = f["O1"] / (f["E0"][:, None] + f["E0"][None, :])
    O2 = W1 @ f["E1p"] - f["E1"] @ W1
    A = W1 @ O2.conj().T
    return 0.5 * (A + A.conj().T)
