"""Picture change of property operators on the GPU (x2c_picture_change
through the C ABI) against the oracle (Eq. utrans with a property's 4c
matrix; U^L = R, U^S = X R).

Inputs of both sides: the oracle's X and R of each block (x2c_direct) and
property matrices from the integral generator.  The GPU forms the same
products in FP64 in another order; the results are compared at 1e-11 of
their largest entry for a multiplicative operator (the nuclear attraction:
P_LL = V, P_SS = W / 4c^2) and at 1e-10 for the Dirac matrix itself, whose
P_SS = W/4c^2 - T cancels to about 1e-1 of its parts.  End to end, the GPU's
own X and R (from x2c_build_batched_xr) must map the identity operator to
the metric S (renormalisation, Eq. ulnonortho, which holds for any X: 2e-9).
"""
import numpy as np
import pytest

import oracle.routes as ox
from x2c_inputs import C_LIGHT as C, atom_block, pack_blocks

pytestmark = pytest.mark.gpu


def _px():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_4446_amd as px
    return px, torch


def _flat(mats, twocomp):
    parts = []
    for M in mats:
        M = np.ascontiguousarray(M, dtype=np.complex128 if twocomp else np.float64)
        parts.append(M.view(np.float64).ravel())
    return np.concatenate(parts)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("twocomp", [False, True])
def test_picture_change_matches_oracle(twocomp):
    px, torch = _px()
    blocks = [atom_block(z) for z in (6, 47, 17)]
    Ns = np.array([b.S.shape[0] for b in blocks], dtype=np.int32)
    n = Ns * (2 if twocomp else 1)
    hsz = n.astype(np.int64) ** 2 * (2 if twocomp else 1)
    p_off = np.concatenate([[0], np.cumsum(hsz)[:-1]]).astype(np.int64)
    Xs, Rs, Vs, Ts, WSs, Dss, refs_v, refs_d = [], [], [], [], [], [], [], []
    for b in blocks:
        W = b.W if twocomp else b.W[0]
        h, _, parts = ox.x2c_direct(b.S, b.T, b.V, W, C, twocomp, return_parts=True)
        Sx, Tx, Vx, Wx = ox.spinor_matrices(b.S, b.T, b.V, W, twocomp)
        PLL, PLS, PSL, PSS = ox.property_blocks(b.V, b.W if twocomp else b.W[0], C, twocomp)
        Xs.append(parts["X"]); Rs.append(parts["R"])
        Vs.append(PLL); Ts.append(Tx); WSs.append(PSS); Dss.append(Wx / (4.0 * C * C) - Tx)
        refs_v.append(ox.picture_change(PLL, PLS, PSL, PSS, parts["X"], parts["R"]))
        refs_d.append(ox.picture_change(Vx, Tx, Tx, Wx / (4.0 * C * C) - Tx, parts["X"], parts["R"]))
    d = lambda mats: _dev(torch, _flat(mats, twocomp))
    X, R = d(Xs), d(Rs)
    print(f"  x2c_picture_change (nuclear attraction) twocomp={twocomp}", flush=True)
    out, ws = px.picture_change(Ns, twocomp, p_off, d(Vs), d(WSs), X, R, c=C)
    torch.cuda.synchronize()
    got = px.unpack_h(out.cpu().numpy(), Ns, twocomp)
    for g, r in zip(got, refs_v):
        assert np.abs(g - r).max() <= 1e-11 * np.abs(r).max()
    print(f"  x2c_picture_change (Dirac matrix) twocomp={twocomp}", flush=True)
    Td = d(Ts)
    out2, _ = px.picture_change(Ns, twocomp, p_off, d(Vs), d(Dss), X, R, PLS=Td, PSL=Td, c=C, workspace=ws)
    torch.cuda.synchronize()
    got2 = px.unpack_h(out2.cpu().numpy(), Ns, twocomp)
    for g, r in zip(got2, refs_d):
        assert np.abs(g - r).max() <= 1e-10 * np.abs(r).max()


@pytest.mark.parametrize("twocomp", [False, True])
def test_identity_maps_to_metric_end_to_end(twocomp):
    px, torch = _px()
    blocks = [atom_block(z) for z in (8, 47)]
    bt = px.batch_to_device(pack_blocks(blocks, twocomp), twocomp)
    print(f"  x2c_build_batched_xr twocomp={twocomp}", flush=True)
    (h, eps, info, X, R), ws = px.build_batched_xr(bt, C)
    h_off, _, _, _ = bt.out_layout()
    S_l, W_l = [], []
    for b in blocks:
        N = b.S.shape[0]
        WO = np.stack([2.0 * b.T, np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))])
        PLL, _, _, PSS = ox.property_blocks(b.S, WO, C, twocomp)
        S_l.append(PLL)
        W_l.append(PSS)
    print(f"  x2c_picture_change (identity) twocomp={twocomp}", flush=True)
    out, _ = px.picture_change(bt.Ns, twocomp, h_off, _dev(torch, _flat(S_l, twocomp)),
                               _dev(torch, _flat(W_l, twocomp)), X, R, c=C, workspace=ws)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    got = px.unpack_h(out.cpu().numpy(), bt.Ns, twocomp)
    for g, Sx in zip(got, S_l):
        assert np.abs(g - Sx).max() <= 2e-9 * np.abs(Sx).max()



def test_time_even_quaternion_products_match_complex_and_oracle():
    """x2c_picture_change_kramers: the nuclear attraction and the Dirac matrix
    (time-even) through the quaternion products give the complex path's and
    the oracle's results; a spin-free call is refused."""
    px, torch = _px()
    blocks = [atom_block(z) for z in (6, 47, 17, 1)]
    Ns = np.array([b.S.shape[0] for b in blocks], dtype=np.int32)
    n = 2 * Ns
    hsz = n.astype(np.int64) ** 2 * 2
    p_off = np.concatenate([[0], np.cumsum(hsz)[:-1]]).astype(np.int64)
    Xs, Rs, Ps, Ss, Ts, Dss, refs_v, refs_d = [], [], [], [], [], [], [], []
    for b in blocks:
        _, _, parts = ox.x2c_direct(b.S, b.T, b.V, b.W, C, True, return_parts=True)
        Sx, Tx, Vx, Wx = ox.spinor_matrices(b.S, b.T, b.V, b.W, True)
        PLL, PLS, PSL, PSS = ox.property_blocks(b.V, b.W, C, True)
        Xs.append(parts["X"]); Rs.append(parts["R"]); Ps.append(PLL); Ss.append(PSS); Ts.append(Tx)
        Dss.append(Wx / (4.0 * C * C) - Tx)
        refs_v.append(ox.picture_change(PLL, PLS, PSL, PSS, parts["X"], parts["R"]))
        refs_d.append(ox.picture_change(Vx, Tx, Tx, Wx / (4.0 * C * C) - Tx, parts["X"], parts["R"]))
    d = lambda mats: _dev(torch, _flat(mats, True))
    X, R, Td = d(Xs), d(Rs), d(Ts)
    print("  x2c_picture_change_kramers (nuclear attraction, Dirac matrix)", flush=True)
    outq, ws = px.picture_change(Ns, True, p_off, d(Ps), d(Ss), X, R, c=C, time_even=True)
    outc, _ = px.picture_change(Ns, True, p_off, d(Ps), d(Ss), X, R, c=C, workspace=ws)
    outd, _ = px.picture_change(Ns, True, p_off, d(Ps), d(Dss), X, R, PLS=Td, PSL=Td, c=C, workspace=ws,
                                time_even=True)
    torch.cuda.synchronize()
    gq = px.unpack_h(outq.cpu().numpy(), Ns, True)
    gc = px.unpack_h(outc.cpu().numpy(), Ns, True)
    gd = px.unpack_h(outd.cpu().numpy(), Ns, True)
    for a, b_, r, dq, rd in zip(gq, gc, refs_v, gd, refs_d):
        assert np.abs(a - r).max() <= 1e-11 * np.abs(r).max()
        assert np.abs(a - b_).max() <= 1e-12 * np.abs(r).max()
        assert np.abs(dq - rd).max() <= 1e-10 * np.abs(rd).max()
    # spin-free blocks have no quaternion form
    with pytest.raises(px.X2CError):
        px.picture_change(Ns, False, p_off, d(Ps), d(Ss), X, R, c=C, time_even=True)
