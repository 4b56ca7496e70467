"""Host-side check of the projector's Zolotarev order selection (no GPU).

The positive-energy projector uses Zolotarev's best rational approximation
of sign(x) on [-1, -l] U [l, 1], with l the gap around -c^2 relative to the
spectral radius.  The kernel tries r = 4, 6, ..., 48 pole pairs, keeps the
smallest r whose error reaches 1e-13 (or the best one when the error stops
improving), and flags the block (info 3) when even the best error is above
1e-11.  This test restates the selection in NumPy (Jacobi elliptic functions
by the arithmetic-geometric mean, as the kernel evaluates them) and checks
that

* the gaps of the workloads' blocks (silver, gold spin-free and
  two-component, the largest spin-free block) give errors far below the
  threshold, and
* gap ratios of 1e-6 and 1e-14 cannot be resolved by any order up to 48, so
  the kernel's threshold flags them.
"""
import numpy as np
import pytest

import oracle
from x2c_inputs import C_LIGHT, ag_2c, atom_block

RMAX = 48
ERR_MAX = 1e-11


def sn_cn(u, ell):
    """Jacobi sn(u, k'), cn(u, k') with modulus k' = sqrt(1 - ell^2), by the
    arithmetic-geometric mean scale (Abramowitz & Stegun 16.4.3), started
    from the complementary modulus ell itself so that moduli close to 1 keep
    full accuracy; also returns K(k') = pi / (2 a_N)."""
    a, b, c = [1.0], [ell], [np.sqrt((1.0 - ell) * (1.0 + ell))]
    while abs(c[-1]) > 1e-17 * a[-1] and len(a) < 64:
        a.append(0.5 * (a[-1] + b[-1]))
        c.append(0.5 * (a[-2] - b[-1]))
        b.append(np.sqrt(a[-2] * b[-1]))
    N = len(a) - 1
    phi = (2.0 ** N) * a[N] * np.asarray(u, dtype=float)
    for n in range(N, 0, -1):
        phi = 0.5 * (phi + np.arcsin(c[n] / a[n] * np.sin(phi)))
    return np.sin(phi), np.cos(phi), np.pi / (2.0 * a[N])


def zolotarev_error(ell: float, r: int) -> float:
    """max |sign(x) - M x (1 + sum_j a_j / (x^2 + c_j))| on [ell, 1], attained
    at x = 1 (equioscillation), for the degree-(2r+1, 2r) Zolotarev
    approximant with c_i = ell^2 sn^2(i K'/(2r+1); k') / cn^2(...), k' =
    sqrt(1 - ell^2)."""
    _, _, K = sn_cn(0.0, ell)
    i = np.arange(1, 2 * r + 1)
    sn, cn, _ = sn_cn(i * K / (2 * r + 1), ell)
    cval = ell * ell * sn * sn / (cn * cn)
    odd, even = cval[0::2], cval[1::2]        # i = 1, 3, ... (poles) and i = 2, 4, ... (zeros)
    a = np.empty(r)
    for j in range(r):
        num = np.prod(even - odd[j])
        den = np.prod(np.delete(odd, j) - odd[j])
        a[j] = num / den
    zhat = lambda x: x * (1.0 + np.sum(a / (x * x + odd)))
    M = 2.0 / (zhat(ell) + zhat(1.0))
    return abs(M * zhat(1.0) - 1.0)


def select(ell: float):
    """The kernel's rule: walk r = 4, 6, ...; keep the best so far; stop at an
    error below 1e-13 or when the error no longer halves."""
    best, best_err, prev = None, None, 1.0
    for r in range(4, RMAX + 1, 2):
        err = zolotarev_error(ell, r)
        if best is None or err <= prev:
            best, best_err = r, err
        if err < 1e-13 or err > 0.5 * prev:
            break
        prev = err
    return best, best_err


def gap_ratio(b, twocomp):
    """0.9 x (distance from -c^2 to the nearest 4c eigenvalue) / (spectral
    radius about -c^2): the kernel's l."""
    import scipy.linalg as sla
    W = b.W if twocomp else b.W[0]
    D, M = oracle.dirac_matrices(*oracle.spinor_matrices(b.S, b.T, b.V, W, twocomp), C_LIGHT)
    e = sla.eigh(D, M, eigvals_only=True)
    sigma = -C_LIGHT ** 2
    gap = min(e[e > sigma].min() - sigma, sigma - e[e < sigma].max())
    radius = max(e.max() - sigma, sigma - e.min())
    return 0.9 * gap / radius


@pytest.mark.parametrize("name,twocomp", [("ag", True), ("Z79", True), ("Z79", False), ("Z1", False)])
def test_workload_gaps_are_resolved(name, twocomp):
    b = ag_2c() if name == "ag" else atom_block(int(name[1:]))
    r, err = select(gap_ratio(b, twocomp))
    assert err < 0.1 * ERR_MAX and r <= RMAX, (name, r, err)


@pytest.mark.parametrize("ell", [1e-6, 1e-14])
def test_tiny_gap_is_flagged(ell):
    r, err = select(ell)
    assert err > ERR_MAX, (r, err)


def test_error_falls_with_order():
    errs = [zolotarev_error(1e-4, r) for r in (4, 8, 12, 16)]
    assert all(b < 0.1 * a for a, b in zip(errs, errs[1:]))
