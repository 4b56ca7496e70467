"""Pins of the BSS and DKHn oracles (oracle/fw.py), CPU only.

Each check is against something other than the oracle's own formulas:
exact decoupling (the positive 4c spectrum), the renormalisation condition
(Eq. renorm), the free-particle closed form, the order of the DKHn error in
the potential, the paper's explicit DKH2 / DKH3 formulas, convergence to
exact decoupling as the order rises, and planted mistakes.
"""
import os

import numpy as np
import pytest

import oracle
import oracle.fw as fw
import oracle.routes as ox
from tests.test_oracle import random_spd_problem
from x2c_inputs import C_LIGHT, atom_block, neon_s20

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dkh_multiplications.txt")

CASES = [
    ("random N=3 two-component, c=7", lambda: random_spd_problem(3, 2, True), 7.0, True),
    ("random N=6 spin-free, c=7", lambda: random_spd_problem(6, 5, False), 7.0, False),
    ("neon s20 spin-free", lambda: (neon_s20().S, neon_s20().T, neon_s20().V, neon_s20().W[0]), C_LIGHT, False),
    ("oxygen two-component", lambda: (atom_block(8).S, atom_block(8).T, atom_block(8).V, atom_block(8).W),
     C_LIGHT, True),
]


def spinor(A, twocomp):
    return oracle.spin_blockdiag(A) if twocomp else np.asarray(A, dtype=float)


# ------------------------------------------------------------------- BSS

@pytest.mark.parametrize("name,make,c,twocomp", CASES)
def test_bss_decouples_exactly(name, make, c, twocomp):
    """eig(h_BSS, S) = the positive-energy 4c spectrum (Sec. II: BSS is an
    exact decoupling of the same 4c problem)."""
    S, T, V, W = make()
    h, eps = fw.bss(S, T, V, W, c, twocomp)
    e4 = oracle.dirac_positive_spectrum(S, T, V, W, c, twocomp)
    es = oracle.spectrum_of(h, S, twocomp)
    assert np.abs(es - e4).max() <= 1e-10 * np.abs(e4).max()
    assert np.abs(eps - e4).max() <= 1e-10 * np.abs(e4).max()
    assert np.abs(h - h.conj().T).max() <= 1e-13 * np.abs(h).max()


@pytest.mark.parametrize("name,make,c,twocomp", CASES)
def test_bss_renormalisation_condition(name, make, c, twocomp):
    """U^L^H S U^L + U^S^H (T/2c^2) U^S = S (Eq. renorm) for the BSS U^L, U^S."""
    S, T, V, W = make()
    _, _, P = fw.bss(S, T, V, W, c, twocomp, return_parts=True)
    Sx, Tx = spinor(S, twocomp), spinor(T, twocomp)
    lhs = P["UL"].conj().T @ Sx @ P["UL"] + P["US"].conj().T @ Tx @ P["US"] / (2 * c * c)
    assert np.abs(lhs - Sx).max() <= 1e-12 * np.abs(Sx).max()


@pytest.mark.parametrize("name,make,c,twocomp", CASES)
def test_bss_utrans_equals_back_transformed_block(name, make, c, twocomp):
    """h from Eq. utrans with U^L_BSS, U^S_BSS equals the electronic block
    of U_1^H H^0 U_1 back-transformed with K^-1 (the paper's two statements
    of the BSS Hamiltonian); this fixes the sign of U^S_BSS."""
    S, T, V, W = make()
    h, _, P = fw.bss(S, T, V, W, c, twocomp, return_parts=True)
    n = P["E1"].shape[0]
    H0, X2, R2 = P["H0"], P["X2"], P["R2"]
    E, O, Ep = H0[:n, :n], H0[:n, n:], H0[n:, n:]
    hp = R2.conj().T @ (E + O @ X2 + X2.conj().T @ O.conj().T + X2.conj().T @ Ep @ X2) @ R2
    hb = fw.back_transform(hp, P["K"])
    assert np.abs(hb - h).max() <= 1e-11 * np.abs(h).max()


def test_bss_printed_small_component_sign_breaks_decoupling():
    """Planted mistake: U^S with (U_0^A X'' - U_0^B), the printed sign, in
    the utrans form no longer gives the 4c spectrum."""
    S, T, V, W = random_spd_problem(4, 3, True)
    c = 7.0
    h, _, P = fw.bss(S, T, V, W, c, True, return_parts=True)
    Sx, Tx, Vx, Wx = oracle.spinor_matrices(S, T, V, W, True)
    UL, US = P["UL"], -P["US"]
    Wp = Wx / (4 * c * c) - Tx
    hm = UL.conj().T @ Vx @ UL + UL.conj().T @ Tx @ US + US.conj().T @ Tx @ UL + US.conj().T @ Wp @ US
    e4 = oracle.dirac_positive_spectrum(S, T, V, W, c, True)
    assert np.abs(oracle.spectrum_of(hm, S, True) - e4).max() > 1e-3 * np.abs(e4).max()


def test_bss_and_x2c_differ_as_matrices_but_not_in_spectrum():
    """Both are exact decouplings of the same 4c problem: same spectrum,
    different (unitarily related) matrices."""
    b = atom_block(8)
    hb, _ = fw.bss(b.S, b.T, b.V, b.W, C_LIGHT, True)
    hx, _ = ox.x2c_direct(b.S, b.T, b.V, b.W, C_LIGHT, True)
    assert np.abs(hb - hx).max() > 1e-8 * np.abs(hx).max()
    e1, e2 = oracle.spectrum_of(hb, b.S, True), oracle.spectrum_of(hx, b.S, True)
    assert np.abs(e1 - e2).max() <= 1e-10 * np.abs(e2).max()


# ------------------------------------------------------------------- DKHn

def free_problem(N=5, seed=3, twocomp=True):
    S, T, V, W = random_spd_problem(N, seed, twocomp)
    return S, T, 0.0 * V, 0.0 * np.asarray(W)


@pytest.mark.parametrize("twocomp", [True, False])
def test_free_particle_closed_form(twocomp):
    """V = W = 0: every DKHn and BSS give h = K^-T (E_0 - c^2) K^-1, whose
    spectrum is 2c^2 t / (sqrt(c^4 + 2c^2 t) + c^2) with T K = S K t."""
    S, T, V, W = free_problem(twocomp=twocomp)
    c = 7.0
    K, t, p = fw.kinetic_basis(S, T)
    ef = 2 * c * c * t / (np.sqrt(c ** 4 + 2 * c * c * t) + c * c)
    Kinv = np.linalg.inv(K)
    href = Kinv.T @ np.diag(ef) @ Kinv
    if twocomp:
        href = oracle.spin_blockdiag(href)
    for n in (1, 2, 3, 5):
        h = fw.dkh(S, T, V, W, c, twocomp, n)
        assert np.abs(h - href).max() <= 1e-12 * np.abs(href).max()
    hb, _ = fw.bss(S, T, V, W, c, twocomp)
    assert np.abs(hb - href).max() <= 1e-12 * np.abs(href).max()


def dkh_error(S, T, V, W, c, twocomp, order, lam):
    """max |eig(h_DKHn) - eig(h_X2C)| with V, W scaled by lam."""
    W = lam * np.asarray(W)
    h = fw.dkh(S, T, lam * V, W, c, twocomp, order)
    hx, _ = ox.x2c_direct(S, T, lam * V, W, c, twocomp)
    return np.abs(oracle.spectrum_of(h, S, twocomp) - oracle.spectrum_of(hx, S, twocomp)).max()


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_dkh_error_is_of_order_n_plus_one(order):
    """DKHn is exact through order n in the potential: halving V and W (at
    small coupling) divides the eigenvalue error by 2^(n+1)."""
    S, T, V, W = random_spd_problem(6, 5, True)
    d1 = dkh_error(S, T, V, W, 7.0, True, order, 0.1)
    d2 = dkh_error(S, T, V, W, 7.0, True, order, 0.05)
    ratio = d1 / d2
    assert 0.75 * 2 ** (order + 1) <= ratio <= 1.3 * 2 ** (order + 1), ratio


def test_dkh_low_orders_match_the_explicit_formulas():
    """The even terms of order 2 and 3 produced by the general algorithm are
    the paper's E_2 = (W_1 O_1^H + c.t.)/2 and E_3 = (W_1 O_2^H + c.t.)/2
    with O_2 = W_1 E_1' - E_1 W_1."""
    S, T, V, W = random_spd_problem(5, 4, True)
    _, P = fw.dkh(S, T, V, W, 7.0, True, 3, return_parts=True)
    n = P["E1"].shape[0]
    E2 = P["terms"][2][:n, :n]
    E3 = P["terms"][3][:n, :n]
    assert np.abs(E2 - fw.dkh2_explicit(P)).max() <= 1e-13 * np.abs(E2).max()
    assert np.abs(E3 - fw.dkh3_explicit(P)).max() <= 1e-13 * np.abs(E3).max()
    # with E_1 and E_1' interchanged inside the bracket the term differs
    W1 = P["O1"] / (P["E0"][:, None] + P["E0"][None, :])
    A = W1 @ (W1 @ P["E1"] - P["E1p"] @ W1).conj().T
    assert np.abs(0.5 * (A + A.conj().T) - E3).max() > 1e-3 * np.abs(E3).max()


def test_dkh_odd_terms_vanish_through_order_n():
    S, T, V, W = random_spd_problem(5, 4, True)
    order = 4
    _, P = fw.dkh(S, T, V, W, 7.0, True, order, return_parts=True)
    n = P["E1"].shape[0]
    sc = np.abs(P["terms"][1]).max()
    for j in range(1, order + 1):
        assert np.abs(P["terms"][j][:n, n:]).max() <= 1e-13 * sc
        assert np.abs(P["terms"][j][n:, :n]).max() <= 1e-13 * sc


def test_dkh_converges_to_exact_decoupling():
    """Bound-state error of DKHn against the 4c spectrum shrinks with every
    order for a copper block (two-component)."""
    b = atom_block(29)
    e4 = oracle.dirac_positive_spectrum(b.S, b.T, b.V, b.W, C_LIGHT, True)
    bd = e4 < 0
    errs = []
    for n in (2, 3, 4, 5, 6):
        h = fw.dkh(b.S, b.T, b.V, b.W, C_LIGHT, True, n)
        errs.append(np.abs(oracle.spectrum_of(h, b.S, True) - e4)[bd].max())
    assert all(b2 < b1 for b1, b2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3 * errs[0]


def test_dkh_planted_mistakes_break_the_order():
    """A wrong commutator coefficient (ad^2 / 1 instead of / 2) or a wrong
    denominator (E_0i + E_0j - c^2) makes DKH2 wrong at second order."""
    S, T, V, W = random_spd_problem(6, 5, True)
    c = 7.0

    def run(mut, lam):
        orig_fact, orig_fp = fw.factorial, fw.fpfw_blocks
        try:
            if mut == "coef":
                fw.factorial = lambda i: 1
            if mut == "denom":
                def fp(*a):
                    f = orig_fp(*a)
                    f = dict(f)
                    f["E0"] = f["E0"] - 0.5 * c * c
                    return f
                fw.fpfw_blocks = fp
            return dkh_error(S, T, V, W, c, True, 2, lam)
        finally:
            fw.factorial, fw.fpfw_blocks = orig_fact, orig_fp

    for mut in ("coef", "denom"):
        ratio = run(mut, 0.1) / run(mut, 0.05)
        assert ratio < 5.0, (mut, ratio)


def test_table_one_counts_are_the_golden_file():
    """The golden fixture holds Table I's 'this work' column."""
    rows = [tuple(map(int, l.split())) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert rows[0] == (2, 1) and rows[1] == (3, 4) and rows[-1] == (14, 266) and len(rows) == 13
