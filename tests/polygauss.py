"""Exact one-centre integrals of (Cartesian polynomial) x exp(-a r^2) functions.

An independent check of the closed forms used by the input generator: basis
functions are written as P(x, y, z) exp(-a r^2) with P a harmonic homogeneous
polynomial (the solid harmonic r^l S_lm built from Legendre polynomials), all
derivatives are taken symbolically on the polynomial, and every integral
reduces to exact sphere moments times radial Gamma functions:

    int x^i y^j z^k dOmega = 2 G((i+1)/2) G((j+1)/2) G((k+1)/2) / G((i+j+k+3)/2)
                             (all exponents even, else 0)
    int_0^inf r^q exp(-p r^2) dr = G((q+1)/2) / (2 p^((q+1)/2))

No formula of the generator is reused here.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly

Poly = dict  # {(i, j, k): complex coefficient}


def padd(*ps):
    out = defaultdict(complex)
    for p in ps:
        for k, v in p.items():
            out[k] += v
    return {k: v for k, v in out.items() if v != 0}


def pscale(p, s):
    return {k: v * s for k, v in p.items()}


def pmul(p, q):
    out = defaultdict(complex)
    for (a, b, c), u in p.items():
        for (d, e, f), v in q.items():
            out[(a + d, b + e, c + f)] += u * v
    return {k: v for k, v in out.items() if v != 0}


def ppow(p, n):
    out = {(0, 0, 0): 1.0 + 0j}
    for _ in range(n):
        out = pmul(out, p)
    return out


def pderiv(p, axis):
    out = defaultdict(complex)
    for key, v in p.items():
        e = key[axis]
        if e == 0:
            continue
        nk = list(key)
        nk[axis] = e - 1
        out[tuple(nk)] += v * e
    return dict(out)


X = {(1, 0, 0): 1.0 + 0j}
Y = {(0, 1, 0): 1.0 + 0j}
Zp = {(0, 0, 1): 1.0 + 0j}
R2 = padd(ppow(X, 2), ppow(Y, 2), ppow(Zp, 2))


def sphere_moment(i, j, k):
    if i % 2 or j % 2 or k % 2:
        return 0.0
    return 2.0 * math.gamma((i + 1) / 2) * math.gamma((j + 1) / 2) * math.gamma((k + 1) / 2) \
        / math.gamma((i + j + k + 3) / 2)


def radial_moment(q, p):
    return math.gamma((q + 1) / 2) / (2.0 * p ** ((q + 1) / 2))


def solid_harmonic_complex(l, m):
    """r^l Y_lm (up to a positive factor), Condon-Shortley phase, as a polynomial.

    For m >= 0:  (-1)^m (x + i y)^m  r^(l-m) P_l^(m)(z/r), where P_l^(m) is the
    m-th derivative of the Legendre polynomial; Y_{l,-m} = (-1)^m conj(Y_lm).
    """
    am = abs(m)
    dP = npleg.legder(npleg.Legendre.basis(l).coef, am)
    pw = npleg.leg2poly(dP)                 # power-basis coefficients in t = z/r
    poly = {}
    for kexp, ck in enumerate(pw):
        if ck == 0:
            continue
        rem = l - am - kexp
        if rem < 0 or rem % 2:
            if abs(ck) > 1e-12 and rem >= 0:
                raise AssertionError("parity violated")
            continue
        term = pmul(ppow(Zp, kexp), ppow(R2, rem // 2))
        poly = padd(poly, pscale(term, ck))
    xpiy = padd(X, pscale(Y, 1j))
    sh = pmul(ppow(xpiy, am), poly)
    sh = pscale(sh, (-1) ** am)
    if m < 0:
        sh = pscale({k: np.conj(v) for k, v in sh.items()}, (-1) ** am)
    return sh


def real_solid_harmonics(l):
    """Real S_lm, m = -l..l, as real polynomials normalised on the sphere."""
    Yc = {m: solid_harmonic_complex(l, m) for m in range(-l, l + 1)}
    # normalise the complex ones on the sphere
    for m in Yc:
        nrm = sphere_integral(pmul(Yc[m], {k: np.conj(v) for k, v in Yc[m].items()}))
        Yc[m] = pscale(Yc[m], 1.0 / math.sqrt(nrm.real))
    s2 = 1.0 / math.sqrt(2.0)
    out = []
    for m in range(-l, l + 1):
        if m == 0:
            p = Yc[0]
        elif m > 0:
            p = padd(pscale(Yc[m], (-1) ** m * s2), pscale(Yc[-m], s2))
        else:
            am = -m
            p = padd(pscale(Yc[-am], 1j * s2), pscale(Yc[am], -1j * (-1) ** am * s2))
        if any(abs(v.imag) > 1e-12 for v in p.values()):
            raise AssertionError("real harmonic has imaginary part")
        out.append({k: v.real + 0j for k, v in p.items() if abs(v) > 1e-15})
    return out


def sphere_integral(p):
    return sum(v * sphere_moment(*k) for k, v in p.items())


def gauss_integral(p, pexp, extra_r_power=0):
    """int P(x,y,z) r^extra exp(-pexp r^2) d^3r for a polynomial P."""
    bydeg = defaultdict(dict)
    for k, v in p.items():
        bydeg[sum(k)][k] = v
    tot = 0j
    for d, part in bydeg.items():
        ang = sphere_integral(part)
        if ang == 0:
            continue
        tot += ang * radial_moment(d + 2 + extra_r_power, pexp)
    return tot


def grad_times_gauss(P, a):
    """Gradient of P exp(-a r^2) = (grad P - 2 a r P) exp(-a r^2): returns the
    three polynomial prefactors."""
    comps = []
    for axis, coord in enumerate((X, Y, Zp)):
        comps.append(padd(pderiv(P, axis), pscale(pmul(coord, P), -2.0 * a)))
    return comps


def one_centre_integrals(funcs, Z):
    """funcs: list of (P, a).  Returns S, T, V, W0, Wx, Wy, Wz (unnormalised)
    by exact polynomial integration:
      S_ij  = int f_i f_j,            T_ij = 1/2 int grad f_i . grad f_j,
      V_ij  = int f_i (-Z/r) f_j,     W0_ij = int (-Z/r) grad f_i . grad f_j,
      Wk_ij = int (-Z/r) (grad f_i x grad f_j)_k.
    """
    n = len(funcs)
    out = {k: np.zeros((n, n)) for k in ("S", "T", "V", "W0", "Wx", "Wy", "Wz")}
    grads = [grad_times_gauss(P, a) for P, a in funcs]
    for i, (Pi, ai) in enumerate(funcs):
        for j, (Pj, aj) in enumerate(funcs):
            p = ai + aj
            gi, gj = grads[i], grads[j]
            out["S"][i, j] = gauss_integral(pmul(Pi, Pj), p).real
            dot = padd(*[pmul(gi[k], gj[k]) for k in range(3)])
            out["T"][i, j] = 0.5 * gauss_integral(dot, p).real
            out["V"][i, j] = -Z * gauss_integral(pmul(Pi, Pj), p, -1).real
            out["W0"][i, j] = -Z * gauss_integral(dot, p, -1).real
            cx = padd(pmul(gi[1], gj[2]), pscale(pmul(gi[2], gj[1]), -1))
            cy = padd(pmul(gi[2], gj[0]), pscale(pmul(gi[0], gj[2]), -1))
            cz = padd(pmul(gi[0], gj[1]), pscale(pmul(gi[1], gj[0]), -1))
            out["Wx"][i, j] = -Z * gauss_integral(cx, p, -1).real
            out["Wy"][i, j] = -Z * gauss_integral(cy, p, -1).real
            out["Wz"][i, j] = -Z * gauss_integral(cz, p, -1).real
    return out
