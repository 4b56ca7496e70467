"""Full-size and maximum-size parity of the HIP path (through the C ABI).

* The Ag309-like batch (309 two-component Z = 47 blocks) in the launch the
  benchmark times (graph replay, four streams), with every product option:
  a seeded sample of blocks against the oracle (strict bound-state limit of
  1e-8 Eh), and for EVERY block the returned eps (from the FP64 eigensolve)
  against the eigenvalues of the returned h with metric S (Eq. 2ceoeq),
  which is where an error of the product chain would show.
* The largest block sizes the library accepts: spin-free N = 512 (real 4c
  dimension 1024), two-component N = 256 with the complex reduction (complex
  4c dimension 1024), and N = 256 with split products.

Tolerances as in tests/test_gpu_parity.py.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from x2c_inputs import C_LIGHT, pack_blocks
from x2c_inputs import integrals as gi
from x2c_inputs.configs import ag309_dlu, shells_for
from tests.test_gpu_parity import DE_BOUND, check_against_oracle, gpu_single

pytestmark = pytest.mark.gpu

PRECS = [0, 1, 2]          # FP64, split bf16, split int8


def _px():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1303_4446_amd as px
    return px, torch


def every_block_eps_vs_h(blocks, hs, eps, twocomp):
    """max over blocks of |eps_GPU - eig(h_GPU, S)| on the bound states, and
    over all states relative to |E|."""
    worst_b = worst_rel = 0.0
    for blk, h, e in zip(blocks, hs, eps):
        Sx = np.kron(np.eye(2), blk.S) if twocomp else blk.S
        es = sla.eigh(0.5 * (h + h.conj().T), Sx, eigvals_only=True)
        d = np.abs(es - e)
        bd = e < 0
        worst_b = max(worst_b, float(d[bd].max()) if bd.any() else 0.0)
        worst_rel = max(worst_rel, float((d / np.maximum(np.abs(e), 1.0)).max()))
    return worst_b, worst_rel


@pytest.mark.parametrize("prec", PRECS)
def test_ag309_full_batch_every_block(prec):
    """The benchmark's batch and launch for each product option."""
    px, torch = _px()
    blocks = ag309_dlu(0)
    pk = pack_blocks(blocks, True)
    bt = px.batch_to_device(pk, True)
    print(f"  ag309 batch prec={prec} (graph replay, 4 streams)", flush=True)
    px.stream_split(4)
    px.graph_enable(True)
    ws = None
    out = None
    for _ in range(2):                     # capture, then replay
        out, ws = px.build_batched(bt, C_LIGHT, prec=prec, workspace=ws, out=out)
    torch.cuda.synchronize()
    h, eps, info = out
    info = info.cpu().numpy()
    assert np.all(info == 0), np.nonzero(info)[0][:10]
    hs = px.unpack_h(h.cpu().numpy(), bt.Ns, True)
    ef = eps.cpu().numpy()
    eps_b = [ef[384 * i:384 * (i + 1)] for i in range(len(blocks))]
    for hb, e in zip(hs, eps_b):
        assert np.abs(hb - hb.conj().T).max() <= 1e-13 * np.abs(hb).max()
        assert np.abs(e[0::2] - e[1::2]).max() <= 1e-12 * np.abs(e).max()
    print("  every block: eps vs eig(h, S)", flush=True)
    wb, wr = every_block_eps_vs_h(blocks, hs, eps_b, True)
    assert wb <= DE_BOUND, f"bound-state |eps - eig(h,S)| {wb:.3e}"
    assert wr <= 1e-10, f"relative |eps - eig(h,S)| {wr:.3e}"
    rng = np.random.default_rng(4321 + prec)
    for i in rng.choice(len(blocks), size=4, replace=False):
        blk = blocks[int(i)]
        print(f"  oracle check block {int(i)} prec={prec}", flush=True)
        check_against_oracle(blk.S, blk.T, blk.V, blk.W, C_LIGHT, True, hs[int(i)], eps_b[int(i)],
                             strict_bound=True)


def _block_of_size(counts, ratio=None, Z=47.0):
    if ratio is None:
        return gi.build_block(Z, shells_for(counts))
    shells = [gi.Shell(l, gi.even_tempered(a0, ratio, counts[l]))
              for l, a0 in ((0, 0.02), (1, 0.03), (2, 0.05), (3, 0.2)) if counts.get(l, 0) > 0]
    return gi.build_block(Z, shells)


def test_spin_free_maximum_block_size():
    """N = 512, the batched limit (spin-free): 32 shells of each l = 0..3 with
    exponent ratio 2 (real 4c dimension 1024)."""
    px, _ = _px()
    N = px.device_wide_min_n(False) - 1
    blk = _block_of_size({0: 32, 1: 32, 2: 32, 3: 32}, ratio=2.0)
    assert blk.N == N == 512
    h, eps = gpu_single(blk.S, blk.T, blk.V, blk.W[0], C_LIGHT, False)
    check_against_oracle(blk.S, blk.T, blk.V, blk.W[0], C_LIGHT, False, h, eps)


@pytest.mark.parametrize("reduction,prec", [(1, 0), (0, 1), (0, 2), (1, 1)])
def test_two_component_maximum_block_size(reduction, prec):
    """N = 256, the batched limit (two-component), with the complex reduction
    (complex 4c dimension 1024) and with split products."""
    px, _ = _px()
    N = px.device_wide_min_n(True) - 1
    blk = _block_of_size({0: 22, 1: 20, 2: 18, 3: 12})
    assert blk.N == N == 256
    h, eps = gpu_single(blk.S, blk.T, blk.V, blk.W, C_LIGHT, True, prec=prec, reduction=reduction)
    check_against_oracle(blk.S, blk.T, blk.V, blk.W, C_LIGHT, True, h, eps)
