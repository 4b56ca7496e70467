"""Pins for the input generator (closed-form one-centre integrals)."""
import math

import numpy as np
import pytest

from x2c_inputs import integrals as gi
from x2c_inputs import configs as cf
from tests import polygauss as pg


def _gen_unnormalised(Z, shells):
    return gi.build_block(Z, shells, normalise=False)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_closed_forms_match_exact_polynomial_integration(l):
    """Generator vs an independent exact polynomial x Gaussian engine:
    S, T, V, W0 and the three spin-orbit matrices, l = 0..3."""
    Z = 7.0
    exps = np.array([0.3, 1.7, 9.0])
    blk = _gen_unnormalised(Z, [gi.Shell(l, exps)])
    harm = pg.real_solid_harmonics(l)
    funcs = []
    for a in exps:
        for P in harm:
            funcs.append((P, float(a)))
    ref = pg.one_centre_integrals(funcs, Z)
    got = dict(S=blk.S, T=blk.T, V=blk.V, W0=blk.W[0], Wx=blk.W[1], Wy=blk.W[2], Wz=blk.W[3])
    for k in ref:
        scale = max(np.abs(ref[k]).max(), 1e-300)
        err = np.abs(got[k] - ref[k]).max() / scale
        assert err < 1e-12, (k, err)
        if l == 0 and k in ("Wx", "Wy", "Wz"):
            assert np.abs(got[k]).max() == 0.0


def test_mixed_shells_block_structure():
    """Two shells together: off-shell-block elements vanish (one centre) and
    the generator's ordering (l, exponent, m) matches the exact engine."""
    Z = 3.0
    shells = [gi.Shell(0, np.array([0.5, 2.0])), gi.Shell(1, np.array([0.8])),
              gi.Shell(2, np.array([1.1]))]
    blk = _gen_unnormalised(Z, shells)
    funcs = []
    for sh in shells:
        harm = pg.real_solid_harmonics(sh.l)
        for a in sh.exponents:
            for P in harm:
                funcs.append((P, float(a)))
    ref = pg.one_centre_integrals(funcs, Z)
    assert np.abs(blk.S - ref["S"]).max() < 1e-13 * np.abs(ref["S"]).max()
    assert np.abs(blk.W[3] - ref["Wz"]).max() < 1e-12 * np.abs(ref["Wz"]).max()
    assert np.abs(blk.W[1] - ref["Wx"]).max() < 1e-12 * np.abs(ref["Wx"]).max()


def test_s_only_forms_of_neon_workload():
    """The four unnormalised s-function forms of the Z=10 workload
    (S=(pi/p)^1.5, T=3ab/p S, V=-2 pi Z/p, W=-8 pi Z ab/p^2) equal the
    generator's radial integrals times 4 pi (angular factor of Y00)."""
    exps = 0.05 * 3.0 ** np.arange(20)
    ref = gi.s_only_block_unnormalised(10.0, exps)
    got = _gen_unnormalised(10.0, [gi.Shell(0, exps)])
    for a, b in ((got.S, ref.S), (got.T, ref.T), (got.V, ref.V), (got.W[0], ref.W[0])):
        assert np.abs(4 * np.pi * a - b).max() <= 1e-14 * np.abs(b).max()


def test_symmetry_and_normalisation():
    blk = cf.ag_2c()
    assert blk.N == 192
    assert np.allclose(np.diag(blk.S), 1.0, atol=0, rtol=0)
    for M in (blk.S, blk.T, blk.V, blk.W[0]):
        assert np.abs(M - M.T).max() <= 1e-15 * np.abs(M).max()
    for k in (1, 2, 3):
        assert np.abs(blk.W[k] + blk.W[k].T).max() <= 1e-15 * np.abs(blk.W[k]).max()
    from oracle import assemble_w
    Wc = assemble_w(*blk.W)
    assert np.abs(Wc - Wc.conj().T).max() <= 1e-15 * np.abs(Wc).max()


def test_angular_momentum_algebra():
    """A^k = <S|(r x grad)_k|S> = i L_k: [A^x, A^y] = -A^z (cyclic),
    sum_k (A^k)^2 = -l(l+1) I, and for l = 1 (order y, z, x) A^k_ij = eps_kij."""
    for l in range(1, 4):
        A = gi.rxgrad_real(l)
        for k in range(3):
            assert np.abs(A[k] + A[k].T).max() < 1e-14
        for (a, b, c) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
            comm = A[a] @ A[b] - A[b] @ A[a]
            assert np.abs(comm + A[c]).max() < 1e-13
        cas = sum(A[k] @ A[k] for k in range(3))
        assert np.abs(cas + l * (l + 1) * np.eye(2 * l + 1)).max() < 1e-12
    A = gi.rxgrad_real(1)
    # real order m=-1,0,1 -> y, z, x ; Cartesian index of each
    cart = {0: 1, 1: 2, 2: 0}
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1
    for k in range(3):
        for i in range(3):
            for j in range(3):
                assert abs(A[k, i, j] - eps[k, cart[i], cart[j]]) < 1e-14


def test_shell_counts():
    N = {Z: cf.atom_block(Z).N for Z in cf.Z_CHOICES}
    assert N == {1: 24, 6: 31, 8: 32, 17: 45, 29: 78, 47: 123, 79: 200}


def test_seeded_workloads_are_deterministic():
    a = cf.ag309_factors(0)
    b = cf.ag309_factors(0)
    assert np.array_equal(a, b) and a.min() >= 0.98 and a.max() <= 1.02
    z0 = [blk.Z for blk in cf.mixed_dlu(1, 32)]
    z1 = [blk.Z for blk in cf.mixed_dlu(1, 32)]
    assert z0 == z1


def test_pack_layout():
    blocks = [cf.atom_block(1), cf.atom_block(6)]
    pk = cf.pack_blocks(blocks, twocomp=True)
    assert list(pk["in_off"]) == [0, 24 * 24]
    o = pk["in_off"][1]
    n2 = 31 * 31
    assert np.array_equal(pk["S"][o:o + n2].reshape(31, 31), blocks[1].S)
    assert np.array_equal(pk["W"][4 * o + 2 * n2:4 * o + 3 * n2].reshape(31, 31), blocks[1].W[2])
