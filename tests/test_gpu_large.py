"""Parity of the device-wide path (one large block on the whole GPU: blocked
Cholesky factors, the positive-energy projector by a Newton-Schulz sign
iteration, X~ and Q^-1/2 by Newton-Schulz iterations) with the CPU oracle,
through the C ABI.

The path runs by default for blocks above the batched limit (N > 256
two-component, > 512 spin-free); x2c_device_wide_min_n lowers the threshold
so that atomic blocks and small molecules, which the oracle solves in
seconds, take it too.

Tolerances are those of the batched path (tests/test_gpu_parity.py): h
elementwise 2e-10 relative to max|h_oracle| (unit roundoff times
kappa(L_T)), bound states of the spectrum of h within 1e-8 Eh of the
oracle's positive 4c eigenvalues (10x the oracle's own floor where that is
larger).  The path does not produce eigenvalues: eps must be NaN.
"""
import contextlib
import os

import numpy as np
import pytest

import oracle
import oracle.routes as ox
from tests.test_oracle import random_spd_problem
from x2c_inputs import C_LIGHT, ag_2c, atom_block, neon_s20, pack_blocks
from x2c_inputs.configs import coupled_molecule

pytestmark = pytest.mark.gpu

TOL_H = 2e-10
DE_BOUND = 1e-8
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ag13_full_seed0.npz")


def _px():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_4446_amd as px
    return px, torch


@contextlib.contextmanager
def device_wide_from(twocomp, n):
    px, _ = _px()
    old = px.device_wide_min_n(twocomp, n)
    try:
        yield
    finally:
        px.device_wide_min_n(twocomp, old)


def gpu_single(S, T, V, W, c, twocomp, prec=0, reduction=0):
    px, torch = _px()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    print(f"  x2c_build N={S.shape[0]} twocomp={twocomp} c={c} prec={prec} reduction={reduction} "
          f"device-wide from {px.device_wide_min_n(twocomp)}", flush=True)
    h, eps = px.build(d(S), d(T), d(V), d(W), c, twocomp, prec=prec, reduction=reduction)
    return h.cpu().numpy(), eps.cpu().numpy()


def check_h(S, T, V, W, c, twocomp, h, strict_bound=False):
    h0, _ = ox.x2c_direct(S, T, V, W, c, twocomp)
    err = np.abs(h - h0).max() / np.abs(h0).max()
    e4 = oracle.dirac_positive_spectrum(S, T, V, W, c, twocomp)
    de = np.abs(oracle.spectrum_of(h, S, twocomp) - e4)
    f = np.abs(oracle.spectrum_of(h0, S, twocomp) - e4)
    bd = e4 < 0
    print(f"    h rel err {err:.2e}; bound dE {de[bd].max() if bd.any() else 0:.2e} "
          f"(oracle floor {f[bd].max() if bd.any() else 0:.2e})", flush=True)
    assert err <= TOL_H, err
    assert np.abs(h - h.conj().T).max() <= 1e-13 * np.abs(h).max()
    if bd.any():
        lim = DE_BOUND if strict_bound else max(DE_BOUND, 10 * f[bd].max())
        assert de[bd].max() <= lim
    return err


@pytest.mark.parametrize("Z,twocomp", [(47, True), (79, True), (17, False), (1, True), (10, False)])
def test_device_wide_atoms_match_oracle(Z, twocomp):
    """Ragged sizes (N = 192, 200, 45, 24, 20: several 64-wide tiles and
    tails, and a single partial tile)."""
    b = neon_s20() if Z == 10 else atom_block(Z)
    W = b.W if twocomp else b.W[0]
    with device_wide_from(twocomp, 1):
        h, eps = gpu_single(b.S, b.T, b.V, W, C_LIGHT, twocomp)
    assert np.all(np.isnan(eps))
    check_h(b.S, b.T, b.V, W, C_LIGHT, twocomp, h, strict_bound=Z == 47)


@pytest.mark.parametrize("N,seed,twocomp", [(1, 0, False), (3, 2, True), (6, 5, False), (1, 7, True),
                                            (40, 3, False), (30, 9, True)])
def test_device_wide_tiny_random(N, seed, twocomp):
    S, T, V, W = random_spd_problem(N, seed, twocomp)
    with device_wide_from(twocomp, 1):
        h, eps = gpu_single(S, T, V, W, 7.0, twocomp)
    check_h(S, T, V, W, 7.0, twocomp, h)


@pytest.mark.parametrize("reduction,prec", [(1, 0), (0, 1), (0, 2), (1, 1)])
def test_device_wide_reductions_and_split_products(reduction, prec):
    """Complex form of the 4c matrix, and the product chain on split bf16 /
    int8 slices (the iterations stay FP64)."""
    b = ag_2c()
    with device_wide_from(True, 1):
        h, eps = gpu_single(b.S, b.T, b.V, b.W, C_LIGHT, True, prec=prec, reduction=reduction)
    check_h(b.S, b.T, b.V, b.W, C_LIGHT, True, h, strict_bound=True)


def test_mixed_batch_device_wide_and_batched_blocks():
    """Blocks at or above the threshold run device-wide (eps NaN), the others
    batched (eps from the eigensolver); every block against the oracle."""
    px, torch = _px()
    blocks = [atom_block(z) for z in (8, 47, 1, 79, 17)]
    with device_wide_from(True, 100):
        bt = px.batch_to_device(pack_blocks(blocks, True), True)
        print(f"  mixed batch N={list(bt.Ns)}", flush=True)
        (h, eps, info), _ = px.build_batched(bt, C_LIGHT)
        torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    hs = px.unpack_h(h.cpu().numpy(), bt.Ns, True)
    e = eps.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(2 * bt.Ns)])
    for i, b in enumerate(blocks):
        ei = e[offs[i]:offs[i + 1]]
        if b.N >= 100:
            assert np.all(np.isnan(ei))
        else:
            e0 = ox.x2c_direct(b.S, b.T, b.V, b.W, C_LIGHT, True)[1]
            assert np.abs(ei - e0).max() <= 1e-12 * np.abs(e0).max()
        check_h(b.S, b.T, b.V, b.W, C_LIGHT, True, hs[i])


@pytest.mark.parametrize("twocomp,reduction", [(True, 0), (False, 0), (True, 1)])
def test_many_blocks_device_wide_in_one_launch_sequence(twocomp, reduction):
    """Every block of a batch of thirteen atoms (seven sizes, in no order)
    forced onto the device-wide path: the blocks run together, each kernel
    covering all of them up to the largest; each block against the oracle."""
    px, torch = _px()
    zs = (47, 1, 8, 79, 17, 10, 47, 6, 1, 36, 8, 79, 55)
    blocks = [atom_block(z) for z in zs]
    with device_wide_from(twocomp, 1):
        bt = px.batch_to_device(pack_blocks(blocks, twocomp), twocomp)
        print(f"  device-wide batch twocomp={twocomp} reduction={reduction} N={list(bt.Ns)}", flush=True)
        (h, eps, info), _ = px.build_batched(bt, C_LIGHT, reduction=reduction)
        torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    assert np.all(np.isnan(eps.cpu().numpy()))
    hs = px.unpack_h(h.cpu().numpy(), bt.Ns, twocomp)
    for i, b in enumerate(blocks):
        W = b.W if twocomp else b.W[0]
        check_h(b.S, b.T, b.V, W, C_LIGHT, twocomp, hs[i])


def test_routes_device_wide_and_auto():
    """X2C_ROUTE_DEVICE_WIDE puts every block on the device-wide path;
    X2C_ROUTE_AUTO does so for a small batch (thirteen silver blocks: eps NaN)
    and keeps the batched path for a large one (309 blocks: eps written).
    h agrees with the size route's and with the oracle."""
    px, torch = _px()
    b = ag_2c()
    h0 = ox.x2c_direct(b.S, b.T, b.V, b.W, C_LIGHT, True)[0]
    bt = px.batch_to_device(pack_blocks([b] * 13, True), True)
    ref = None
    for route in (px.ROUTE_SIZE, px.ROUTE_DEVICE_WIDE, px.ROUTE_AUTO):
        print(f"  13 silver blocks, route {route}", flush=True)
        (h, eps, info), _ = px.build_batched(bt, C_LIGHT, route=route)
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        assert bool(torch.isnan(eps).all()) == (route != px.ROUTE_SIZE)
        hs = px.unpack_h(h.cpu().numpy(), bt.Ns, True)
        for hb in hs:
            assert np.abs(hb - h0).max() <= TOL_H * np.abs(h0).max()
        if ref is None:
            ref = hs[0]
        else:
            assert np.abs(hs[0] - ref).max() <= TOL_H * np.abs(ref).max()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    print("  one silver block, x2c_build, route auto", flush=True)
    h1, e1 = px.build(d(b.S), d(b.T), d(b.V), d(b.W), C_LIGHT, True, route=px.ROUTE_AUTO)
    assert bool(torch.isnan(e1).all())
    assert np.abs(h1.cpu().numpy() - h0).max() <= TOL_H * np.abs(h0).max()
    big = px.batch_to_device(pack_blocks([b] * 309, True), True)
    print("  309 silver blocks, route auto", flush=True)
    (h, eps, info), _ = px.build_batched(big, C_LIGHT, route=px.ROUTE_AUTO)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    assert bool(torch.isfinite(eps).all())
    hl = px.unpack_h(h.cpu().numpy(), big.Ns, True)
    for i in (0, 154, 308):
        assert np.abs(hl[i] - h0).max() <= TOL_H * np.abs(h0).max()
    sf = [atom_block(z) for z in (79, 36, 8)]
    bs = px.batch_to_device(pack_blocks(sf, False), False)
    print("  spin-free atoms, route auto", flush=True)
    (h, eps, info), _ = px.build_batched(bs, C_LIGHT, route=px.ROUTE_AUTO)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0) and bool(torch.isnan(eps).all())
    hs = px.unpack_h(h.cpu().numpy(), bs.Ns, False)
    for i, a in enumerate(sf):
        check_h(a.S, a.T, a.V, a.W[0], C_LIGHT, False, hs[i])


def test_device_wide_failure_codes():
    """S or T not positive definite: the blocked factorisation reports the
    batched path's codes (1, 2), h zero."""
    px, torch = _px()
    b = atom_block(8)
    with device_wide_from(True, 1):
        for which, code in (("S", 1), ("T", 2)):
            S, T = b.S.copy(), b.T.copy()
            M = S if which == "S" else T
            M[3, 3] = -abs(M[3, 3])
            d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
            print(f"  device-wide build with {which} not SPD", flush=True)
            with pytest.raises(px.X2CError) as ex:
                px.build(d(S), d(T), d(b.V), d(b.W), C_LIGHT, True)
            assert ex.value.info == code


def test_three_atom_molecule_default_threshold():
    """A coupled three-atom silver molecule (N = 576 > 256): the device-wide
    path by default; h against the oracle's full (non-local) transformation."""
    mol = coupled_molecule([ag_2c() for _ in range(3)], 0)
    px, _ = _px()
    assert mol.Ntot >= px.device_wide_min_n(True)
    h, eps = gpu_single(mol.S, mol.T, mol.V, mol.W, C_LIGHT, True)
    assert np.all(np.isnan(eps))
    check_h(mol.S, mol.T, mol.V, mol.W, C_LIGHT, True, h, strict_bound=True)


def test_spin_free_molecule_above_batched_limit():
    """Spin-free: three coupled silver blocks (N = 576 > 512)."""
    mol = coupled_molecule([ag_2c() for _ in range(3)], 1)
    W0 = mol.W[0]
    h, eps = gpu_single(mol.S, mol.T, mol.V, W0, C_LIGHT, False)
    assert np.all(np.isnan(eps))
    check_h(mol.S, mol.T, mol.V, W0, C_LIGHT, False, h, strict_bound=True)


def test_molecule_and_atoms_device_wide_in_one_batch():
    """A block above the batched limit (three coupled silver atoms, N = 576)
    and two atoms (N = 24, 123) on the device-wide path in one call (the
    route option puts the atoms there): each kernel covers all three, the
    atoms' tiles stop at their own sizes; every block against the oracle."""
    px, torch = _px()
    from x2c_inputs.configs import AtomBlock
    mol = coupled_molecule([ag_2c() for _ in range(3)], 0)
    blocks = [atom_block(1), AtomBlock(47, mol.S, mol.T, mol.V, mol.W), atom_block(47)]
    bt = px.batch_to_device(pack_blocks(blocks, True), True)
    print(f"  device-wide batch N={list(bt.Ns)} (route device-wide)", flush=True)
    (h, eps, info), _ = px.build_batched(bt, C_LIGHT, route=px.ROUTE_DEVICE_WIDE)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    assert bool(torch.isnan(eps).all())
    hs = px.unpack_h(h.cpu().numpy(), bt.Ns, True)
    for i, b in enumerate(blocks):
        check_h(b.S, b.T, b.V, b.W, C_LIGHT, True, hs[i], strict_bound=(i == 1))


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="Ag13 reference not generated")
@pytest.mark.timeout(400)
def test_ag13_full_build_matches_oracle_reference():
    """The full (non-local) two-component X2C of the 13-atom silver molecule
    (N = 2496, 4c dimension 9984 complex) on one GPU, against values the
    oracle wrote (tests/golden/make_ag13_full_reference.py): h applied to a
    seeded block of vectors, five full rows of h, and the bound-state
    spectrum of h against the oracle's positive 4c eigenvalues."""
    import scipy.linalg as sla
    from x2c_inputs.configs import ag13_molecule
    ref = np.load(GOLDEN)
    mol = ag13_molecule(0)
    assert abs(mol.scale - float(ref["coupling_scale"])) == 0.0
    h, eps = gpu_single(mol.S, mol.T, mol.V, mol.W, C_LIGHT, True)
    assert np.all(np.isnan(eps))
    hmax = float(ref["hmax"])
    err_rows = np.abs(h[ref["row_index"]] - ref["rows"]).max() / hmax
    V = ref["V"]
    err_probe = np.abs(h @ V - ref["probes"]).max() / np.abs(ref["probes"]).max()
    print(f"    rows rel err {err_rows:.2e}; h V rel err {err_probe:.2e}", flush=True)
    assert err_rows <= TOL_H
    assert err_probe <= TOL_H
    assert np.abs(h - h.conj().T).max() <= 1e-13 * hmax
    e4 = ref["e4"]
    nb = int((e4 < 0).sum())
    S2 = ox.spin_blockdiag(mol.S)
    es = sla.eigh(0.5 * (h + h.conj().T), S2, eigvals_only=True, subset_by_index=[0, nb - 1])
    de = np.abs(es - e4[:nb]).max()
    print(f"    bound states {nb}: max dE {de:.2e} Eh", flush=True)
    assert de <= DE_BOUND


def _uncoupled(blocks):
    """Block-diagonal molecular S, T, V, W^q of the given atomic blocks (no
    inter-atomic coupling)."""
    Ns = [b.N for b in blocks]
    Nt = int(sum(Ns))
    S = np.zeros((Nt, Nt)); T = np.zeros((Nt, Nt)); V = np.zeros((Nt, Nt)); W = np.zeros((4, Nt, Nt))
    o = 0
    for b in blocks:
        sl = slice(o, o + b.N)
        S[sl, sl] = b.S; T[sl, sl] = b.T; V[sl, sl] = b.V; W[:, sl, sl] = b.W
        o += b.N
    return S, T, V, W, Ns


@pytest.mark.parametrize("twocomp", [True, False])
@pytest.mark.timeout(400)
def test_maximum_size_uncoupled_molecule(twocomp):
    """N = x2c_max_n (4096 two-component, 8192 spin-free): a block-diagonal
    molecule of silver blocks and one block of another size.  The full
    transformation of uncoupled atoms is the direct sum of the atomic ones
    (Sec. III.A: the DLU approximation is exact then), so every diagonal
    block must equal the oracle's atomic h and every other entry vanish."""
    px, _ = _px()
    from tests.test_gpu_fullsize import _block_of_size
    Nmax = px.max_n(twocomp)
    extra = _block_of_size({0: 22, 1: 20, 2: 18, 3: 12}) if twocomp else _block_of_size({0: 24, 1: 12, 2: 8, 3: 4})
    ag = ag_2c()
    k = (Nmax - extra.N) // ag.N
    blocks = [ag] * (k // 2) + [extra] + [ag] * (k - k // 2)
    S, T, V, W, Ns = _uncoupled(blocks)
    assert S.shape[0] == Nmax
    Wm = W if twocomp else W[0]
    h, eps = gpu_single(S, T, V, Wm, C_LIGHT, twocomp)
    assert np.all(np.isnan(eps))
    refs = {}
    for b in (ag, extra):
        Wb = b.W if twocomp else b.W[0]
        refs[id(b)] = ox.x2c_direct(b.S, b.T, b.V, Wb, C_LIGHT, twocomp)[0]
    hmax = max(np.abs(r).max() for r in refs.values())
    mask = np.zeros(h.shape, dtype=bool)
    o = 0
    worst = 0.0
    for b in blocks:
        idx = ox.atom_spinor_index(o, b.N, Nmax, twocomp)
        r = refs[id(b)]
        worst = max(worst, np.abs(h[np.ix_(idx, idx)] - r).max() / np.abs(r).max())
        mask[np.ix_(idx, idx)] = True
        o += b.N
    off = np.abs(h[~mask]).max()
    print(f"    N={Nmax}: diagonal blocks rel err {worst:.2e}; largest off-block entry {off:.2e} "
          f"(max|h| {hmax:.2e})", flush=True)
    assert worst <= TOL_H
    assert off <= 1e-13 * hmax


def test_device_wide_reproducible_and_graph_replays_match_eager():
    """The device-wide path sums its convergence measures in a fixed order:
    two eager calls and two graph replays (same buffers, unrelated eager
    work in between) give the same bits."""
    px, torch = _px()
    blocks = [atom_block(47)]
    with device_wide_from(True, 1):
        bt = px.batch_to_device(pack_blocks(blocks, True), True)
        h_off, eps_off, hsz, esz = bt.out_layout()
        out = (torch.empty(hsz, dtype=torch.float64, device="cuda"),
               torch.empty(esz, dtype=torch.float64, device="cuda"),
               torch.empty(1, dtype=torch.int32, device="cuda"))
        ws = None
        got = []
        prev = px.graph_enable(False)
        try:
            for graph in (False, False, True, True):
                px.graph_enable(graph)
                junk = torch.randn(1 << 20, device="cuda").sum()
                print(f"  device-wide build, graph={graph}", flush=True)
                (h, eps, info), ws = px.build_batched(bt, C_LIGHT, workspace=ws, out=out)
                torch.cuda.synchronize()
                assert float(junk) == float(junk)
                assert int(info.cpu()[0]) == 0
                got.append(h.cpu().numpy().copy())
        finally:
            px.graph_enable(prev)
    for g in got[1:]:
        assert np.array_equal(g, got[0])


def test_device_wide_x_r_outputs_and_picture_change():
    """x2c_build_batched_xr on a block above the batched limit (three coupled
    silver atoms, N = 576): X and R against the oracle's (2e-9, u times the
    conditioning of the X formula; the Newton-Schulz route's rounding stays
    below it), and the picture change of the nuclear
    attraction with the GPU's X and R, complex and quaternion products,
    against the oracle's formula with its own X and R."""
    px, torch = _px()
    mol = coupled_molecule([ag_2c() for _ in range(3)], 2)
    from x2c_inputs import pack_blocks as pk_
    from x2c_inputs.configs import AtomBlock
    blk = AtomBlock(47, mol.S, mol.T, mol.V, mol.W)
    bt = px.batch_to_device(pk_([blk], True), True)
    print(f"  x2c_build_batched_xr N={mol.Ntot}", flush=True)
    (h, eps, info, X, R), ws = px.build_batched_xr(bt, C_LIGHT)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    Xg = px.unpack_h(X.cpu().numpy(), bt.Ns, True)[0]
    Rg = px.unpack_h(R.cpu().numpy(), bt.Ns, True)[0]
    _, _, parts = ox.x2c_direct(mol.S, mol.T, mol.V, mol.W, C_LIGHT, True, return_parts=True)
    ex = np.abs(Xg - parts["X"]).max() / np.abs(parts["X"]).max()
    er = np.abs(Rg - parts["R"]).max() / np.abs(parts["R"]).max()
    print(f"    X rel err {ex:.2e}, R rel err {er:.2e}", flush=True)
    assert ex <= 2e-9 and er <= 2e-9
    PLL, PLS, PSL, PSS = ox.property_blocks(mol.V, mol.W, C_LIGHT, True)
    ref = ox.picture_change(PLL, PLS, PSL, PSS, parts["X"], parts["R"])
    h_off = bt.out_layout()[0]
    flat = lambda M: torch.from_numpy(np.ascontiguousarray(M, dtype=np.complex128).view(np.float64).ravel()).cuda()
    for even in (False, True):
        print(f"  picture change time_even={even}", flush=True)
        out, _ = px.picture_change(bt.Ns, True, h_off, flat(PLL), flat(PSS), X, R, c=C_LIGHT, time_even=even)
        torch.cuda.synchronize()
        got = px.unpack_h(out.cpu().numpy(), bt.Ns, True)[0]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"    picture change rel err {err:.2e}", flush=True)
        assert err <= 1e-9


def test_device_wide_failure_codes_in_one_batch():
    """Blocks forced onto the device-wide path fail as on the batched path:
    S or T not positive definite (1, 2), non-finite input (6), a singular S
    (duplicated function, 1); their h and eps are zero, the good blocks are
    unaffected.  c = 1 with Z = 79 leaves no gap at -c^2: the sign iteration
    cannot converge or splits the spectrum unevenly (3 or 4)."""
    px, torch = _px()
    from x2c_inputs.integrals import AtomBlock
    good = atom_block(8)

    def mod(**kw):
        d = dict(Z=good.Z, S=good.S.copy(), T=good.T.copy(), V=good.V.copy(), W=good.W.copy())
        d.update(kw)
        return AtomBlock(**d)

    sbad = good.S.copy(); sbad[3, 3] = -1.0
    tbad = good.T.copy(); tbad[2, 2] = -5.0
    vnan = good.V.copy(); vnan[1, 4] = np.nan; vnan[4, 1] = np.nan
    dup = neon_s20()
    Sd, Td, Vd, Wd = dup.S.copy(), dup.T.copy(), dup.V.copy(), dup.W.copy()
    for M in (Sd, Td, Vd, Wd[0]):
        M[1, :] = M[0, :]; M[:, 1] = M[:, 0]
    blocks = [good, mod(S=sbad), mod(T=tbad), mod(V=vnan), AtomBlock(Z=10.0, S=Sd, T=Td, V=Vd, W=Wd), good]
    for twocomp in (False, True):
        with device_wide_from(twocomp, 1):
            bt = px.batch_to_device(pack_blocks(blocks, twocomp), twocomp)
            print(f"  device-wide failure batch twocomp={twocomp}", flush=True)
            (h, eps, info), _ = px.build_batched(bt, C_LIGHT)
            torch.cuda.synchronize()
        info = list(info.cpu().numpy())
        assert info == [0, 1, 2, 6, 1, 0], info
        hs = px.unpack_h(h.cpu().numpy(), bt.Ns, twocomp)
        e = eps.cpu().numpy()
        offs = np.concatenate([[0], np.cumsum(bt.Ns * (2 if twocomp else 1))])
        for i in (1, 2, 3, 4):
            assert not np.any(hs[i]) and not np.any(e[offs[i]:offs[i + 1]])
        W = good.W if twocomp else good.W[0]
        h0 = ox.x2c_direct(good.S, good.T, good.V, W, C_LIGHT, twocomp)[0]
        for i in (0, 5):
            assert np.abs(hs[i] - h0).max() <= TOL_H * np.abs(h0).max()
    blk = atom_block(79)
    with device_wide_from(False, 1):
        bt = px.batch_to_device(pack_blocks([blk, atom_block(1)], False), False)
        print("  device-wide branch failure (Z = 79, c = 1)", flush=True)
        (h, eps, info), _ = px.build_batched(bt, 1.0)
        torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[0] in (3, 4), info
    assert not np.any(px.unpack_h(h.cpu().numpy(), bt.Ns, False)[0])
