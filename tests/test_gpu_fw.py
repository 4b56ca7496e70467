"""Parity of the HIP BSS and DKHn paths (x2c_bss_batched, x2c_dkh_batched,
through the C ABI) with the CPU oracle (oracle/fw.py).

Tolerances:
  * h elementwise: |h - h_oracle| <= TOL_H_FW * max|h_oracle|.  Both sides
    build the kinetic basis K from T K = S K t (different eigenvector
    routines: LAPACK against tridiagonal QR on the GPU; h does not depend on
    the choice inside degenerate eigenspaces).  Every step is backward stable
    in ||C|| = ||L_S^-1 T L_S^-T||; the back-transformation with S K carries
    kappa(S) (<= 1e5 for these bases): u kappa(S) ~ 1e-11, so 1e-10 is the
    FP64 bar.  BSS additionally takes X from the X2C solve (its forward error
    2e-9 relative, the X tolerance of the X2C tests), so its h is held to
    2e-9.
  * BSS spectrum: eig(h, S) against the oracle's positive 4c spectrum, bound
    states <= 1e-8 Eh (exact decoupling).
"""
import numpy as np
import pytest

import oracle
import oracle.fw as fw
from tests.test_oracle import random_spd_problem
from x2c_inputs import C_LIGHT, atom_block, neon_s20, pack_blocks
from x2c_inputs.configs import ag309_dlu

pytestmark = pytest.mark.gpu

TOL_H_FW = 1e-10
TOL_H_BSS = 2e-9
DE_BOUND = 1e-8


def _px():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_4446_amd as px
    return px, torch


class Blk:
    def __init__(self, S, T, V, W):
        self.S, self.T, self.V = S, T, V
        W = np.asarray(W)
        self.W = W if W.ndim == 3 else W[None]
        self.N = S.shape[0]


def gpu_run(blocks, twocomp, c, method, order=0):
    px, torch = _px()
    bt = px.batch_to_device(pack_blocks(blocks, twocomp), twocomp)
    print(f"  {method} order={order} nblk={len(blocks)} N={list(bt.Ns)[:8]} twocomp={twocomp} c={c}", flush=True)
    if method == "dkh":
        (h, info), _ = px.dkh_batched(bt, c, order)
        eps = None
    else:
        (h, eps, info), _ = px.bss_batched(bt, c)
    torch.cuda.synchronize()
    hs = px.unpack_h(h.cpu().numpy(), bt.Ns, twocomp)
    info = info.cpu().numpy()
    if eps is not None:
        n = bt.Ns * (2 if twocomp else 1)
        offs = np.concatenate([[0], np.cumsum(n)])
        e = eps.cpu().numpy()
        eps = [e[offs[i]:offs[i + 1]] for i in range(len(blocks))]
    return hs, eps, info


def wmat(b, twocomp):
    return b.W if twocomp else b.W[0]


def check_dkh(b, twocomp, c, order, h):
    h0 = fw.dkh(b.S, b.T, b.V, wmat(b, twocomp), c, twocomp, order)
    err = np.abs(h - h0).max() / np.abs(h0).max()
    print(f"    DKH{order} h rel err {err:.2e}", flush=True)
    assert err <= TOL_H_FW, err
    assert np.abs(h - h.conj().T).max() <= 1e-13 * np.abs(h).max()
    return err


def check_bss(b, twocomp, c, h, eps, strict=False):
    W = wmat(b, twocomp)
    h0, e0 = fw.bss(b.S, b.T, b.V, W, c, twocomp)
    err = np.abs(h - h0).max() / np.abs(h0).max()
    e4 = oracle.dirac_positive_spectrum(b.S, b.T, b.V, W, c, twocomp)
    es = oracle.spectrum_of(h, b.S, twocomp)
    f = np.abs(oracle.spectrum_of(h0, b.S, twocomp) - e4)
    de = np.abs(es - e4)
    bd = e4 < 0
    print(f"    BSS h rel err {err:.2e}; bound dE {de[bd].max() if bd.any() else 0:.2e} "
          f"(oracle floor {f[bd].max() if bd.any() else 0:.2e})", flush=True)
    assert err <= TOL_H_BSS, err
    assert np.abs(eps - e0).max() <= 1e-12 * np.abs(e0).max()
    if bd.any():
        lim = DE_BOUND if strict else max(DE_BOUND, 10 * f[bd].max())
        assert de[bd].max() <= lim
    assert np.all(de <= np.maximum(max(DE_BOUND, 10 * f.max()), 1e-12 * np.abs(e4)))
    return err


# ------------------------------------------------------------------- DKHn

@pytest.mark.parametrize("N,seed,twocomp", [(1, 0, False), (3, 2, True), (6, 5, False), (5, 4, True)])
def test_dkh_tiny_random(N, seed, twocomp):
    S, T, V, W = random_spd_problem(N, seed, twocomp)
    b = Blk(S, T, V, W)
    for order in (1, 2, 3, 5):
        hs, _, info = gpu_run([b], twocomp, 7.0, "dkh", order)
        assert np.all(info == 0)
        check_dkh(b, twocomp, 7.0, order, hs[0])


@pytest.mark.parametrize("order", [2, 3, 4, 6, 8])
def test_dkh_atoms_batched(order):
    """Uneven two-component batch (ragged tiles): every block against the oracle."""
    blocks = [atom_block(z) for z in (8, 1, 29, 17)]
    hs, _, info = gpu_run(blocks, True, C_LIGHT, "dkh", order)
    assert np.all(info == 0)
    for b, h in zip(blocks, hs):
        check_dkh(b, True, C_LIGHT, order, h)


@pytest.mark.parametrize("order", [2, 4])
def test_dkh_spin_free(order):
    blocks = [neon_s20(), atom_block(47), atom_block(79)]
    sf = [Blk(b.S, b.T, b.V, b.W[0]) for b in blocks]
    hs, _, info = gpu_run(sf, False, C_LIGHT, "dkh", order)
    assert np.all(info == 0)
    for b, h in zip(sf, hs):
        check_dkh(b, False, C_LIGHT, order, h)


def test_dkh_converges_towards_the_dirac_spectrum_on_gpu():
    """GPU DKHn bound-state spectrum approaches the 4c one as n rises."""
    b = atom_block(47)
    e4 = oracle.dirac_positive_spectrum(b.S, b.T, b.V, b.W, C_LIGHT, True)
    bd = e4 < 0
    errs = []
    for order in (2, 4, 6, 8):
        hs, _, info = gpu_run([b], True, C_LIGHT, "dkh", order)
        assert np.all(info == 0)
        errs.append(np.abs(oracle.spectrum_of(hs[0], b.S, True) - e4)[bd].max())
    print(f"    bound-state |dE| by order: {errs}", flush=True)
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))


def test_dkh_ag309_batch_sampled():
    """The Ag309-like batch with DKH2 and DKH4: Kramers-structured Hermitian
    h for every block, a seeded sample against the oracle."""
    blocks = ag309_dlu(0)
    rng = np.random.default_rng(99)
    pick = rng.choice(len(blocks), size=3, replace=False)
    for order in (2, 4):
        hs, _, info = gpu_run(blocks, True, C_LIGHT, "dkh", order)
        assert np.all(info == 0)
        for h in hs:
            assert np.abs(h - h.conj().T).max() <= 1e-13 * np.abs(h).max()
        for i in pick:
            check_dkh(blocks[int(i)], True, C_LIGHT, order, hs[int(i)])


def test_dkh_largest_blocks():
    px, _ = _px()
    from tests.test_gpu_fullsize import _block_of_size
    b2 = _block_of_size({0: 22, 1: 20, 2: 18, 3: 12})
    hs, _, info = gpu_run([b2], True, C_LIGHT, "dkh", 3)
    assert np.all(info == 0)
    check_dkh(b2, True, C_LIGHT, 3, hs[0])
    b1 = _block_of_size({0: 32, 1: 32, 2: 32, 3: 32}, ratio=2.0)
    sf = Blk(b1.S, b1.T, b1.V, b1.W[0])
    hs, _, info = gpu_run([sf], False, C_LIGHT, "dkh", 3)
    assert np.all(info == 0)
    check_dkh(sf, False, C_LIGHT, 3, hs[0])


# ------------------------------------------------------------------- BSS

@pytest.mark.parametrize("N,seed,twocomp", [(1, 0, False), (3, 2, True), (6, 5, False), (5, 4, True)])
def test_bss_tiny_random(N, seed, twocomp):
    S, T, V, W = random_spd_problem(N, seed, twocomp)
    b = Blk(S, T, V, W)
    hs, eps, info = gpu_run([b], twocomp, 7.0, "bss")
    assert np.all(info == 0)
    check_bss(b, twocomp, 7.0, hs[0], eps[0])


def test_bss_atoms_batched():
    blocks = [atom_block(z) for z in (8, 79, 1, 47, 29)]
    hs, eps, info = gpu_run(blocks, True, C_LIGHT, "bss")
    assert np.all(info == 0)
    for b, h, e in zip(blocks, hs, eps):
        check_bss(b, True, C_LIGHT, h, e, strict=b.Z == 47)


def test_bss_spin_free():
    blocks = [neon_s20(), atom_block(79), atom_block(17)]
    sf = [Blk(b.S, b.T, b.V, b.W[0]) for b in blocks]
    hs, eps, info = gpu_run(sf, False, C_LIGHT, "bss")
    assert np.all(info == 0)
    for b, h, e in zip(sf, hs, eps):
        check_bss(b, False, C_LIGHT, h, e)


def test_bss_ag309_batch_sampled():
    blocks = ag309_dlu(0)
    hs, eps, info = gpu_run(blocks, True, C_LIGHT, "bss")
    assert np.all(info == 0)
    for h in hs:
        assert np.abs(h - h.conj().T).max() <= 1e-13 * np.abs(h).max()
    rng = np.random.default_rng(98)
    for i in rng.choice(len(blocks), size=3, replace=False):
        check_bss(blocks[int(i)], True, C_LIGHT, hs[int(i)], eps[int(i)], strict=True)


def test_bss_rejects_split_and_complex_reduction():
    px, torch = _px()
    import ctypes
    from paper_1303_4446_amd import _lib
    lib = px.load()
    N = (ctypes.c_int * 1)(10)
    assert lib.x2c_bss_workspace_bytes(ctypes.byref(_lib.options(True, 137.0, prec=px.SPLIT_BF16)), 1, N) == 0
    assert lib.x2c_bss_workspace_bytes(ctypes.byref(_lib.options(True, 137.0, reduction=px.RED_COMPLEX)), 1, N) == 0
    assert lib.x2c_dkh_workspace_bytes(ctypes.byref(_lib.options(True, 137.0, prec=px.SPLIT_INT8)), 2, 1, N) == 0
