"""Pins of the oracle's DLU molecular Hamiltonian (Sec. III.A, Eqs. dlutrans,
r2ctransatom, utrans) against facts fixed by the definition:

* one atom: DLU is the full transformation (x2c_direct);
* uncoupled atoms: U is then exactly block diagonal, so DLU equals the full
  molecular X2C and every atomic diagonal block equals the atom's own h;
* coupled atoms: the atomic diagonal blocks of h still equal the atoms' h
  (U is block diagonal and the diagonal blocks of S, T, V, W are atomic);
  the DLU error against the full transformation shrinks faster than the
  coupling itself;
* c -> infinity: h -> T + V;
* h is Hermitian.
Planted mistakes in the assembly must fail at least one pin."""
import numpy as np
import pytest

import oracle
import oracle.routes as ox
from x2c_inputs import C_LIGHT as C, atom_block, coupled_molecule

BLOCKS = (1, 8, 6)


def _mol(scale=1e-3, seed=0):
    return coupled_molecule([atom_block(z) for z in BLOCKS], seed, scale=scale)


def _W(m, twocomp):
    return m.W if twocomp else m.W[0]


def _dlu(m, twocomp, c=C):
    return ox.x2c_dlu(m.S, m.T, m.V, _W(m, twocomp), m.Ns, c, twocomp)


@pytest.mark.parametrize("twocomp", [False, True])
def test_dlu_single_atom_is_the_full_transformation(twocomp):
    b = atom_block(8)
    W = b.W if twocomp else b.W[0]
    h = ox.x2c_dlu(b.S, b.T, b.V, W, [b.N], C, twocomp)
    h0, _ = ox.x2c_direct(b.S, b.T, b.V, W, C, twocomp)
    assert np.abs(h - h0).max() <= 1e-13 * np.abs(h0).max()


@pytest.mark.parametrize("twocomp", [False, True])
def test_dlu_uncoupled_equals_full_molecular(twocomp):
    m = _mol(scale=0.0)
    h = _dlu(m, twocomp)
    hf, _ = ox.x2c_direct(m.S, m.T, m.V, _W(m, twocomp), C, twocomp)
    assert np.abs(h - hf).max() <= 1e-12 * np.abs(hf).max()


@pytest.mark.parametrize("twocomp", [False, True])
def test_dlu_atomic_diagonal_blocks_and_hermiticity(twocomp):
    m = _mol()
    h = _dlu(m, twocomp)
    s = np.abs(h).max()
    assert np.abs(h - h.conj().T).max() <= 1e-13 * s
    for A in range(len(BLOCKS)):
        a = m.atom(A)
        W = a.W if twocomp else a.W[0]
        ha, _ = ox.x2c_direct(a.S, a.T, a.V, W, C, twocomp)
        idx = ox.atom_spinor_index(int(m.off[A]), a.N, m.Ntot, twocomp)
        assert np.abs(h[np.ix_(idx, idx)] - ha).max() <= 1e-12 * np.abs(ha).max()
    # the coupling does reach the off-diagonal atom blocks
    i0 = ox.atom_spinor_index(0, int(m.Ns[0]), m.Ntot, twocomp)
    i1 = ox.atom_spinor_index(int(m.off[1]), int(m.Ns[1]), m.Ntot, twocomp)
    assert np.abs(h[np.ix_(i0, i1)]).max() > 1e-6 * s


def test_dlu_error_shrinks_faster_than_the_coupling():
    errs = []
    for sc in (1e-3, 1e-4):
        m = _mol(scale=sc)
        h = _dlu(m, True)
        hf, _ = ox.x2c_direct(m.S, m.T, m.V, m.W, C, True)
        e1 = oracle.spectrum_of(h, m.S, True)
        e2 = oracle.spectrum_of(hf, m.S, True)
        errs.append(np.abs(e1 - e2)[e2 < 0].max())
    assert errs[0] > 0 and errs[1] < errs[0] / 10.0, errs


def test_dlu_nonrelativistic_limit():
    m = _mol()
    TV = m.T + m.V
    r = [np.abs(_dlu(m, False, c=c) - TV).max() / np.abs(TV).max() for c in (1e5, 1e6)]
    assert r[0] < 1e-5 and 50.0 < r[0] / r[1] < 200.0, r


# ---------------------------------------------------------------- planted mistakes

def _pins_pass():
    try:
        b = atom_block(8)
        h = ox.x2c_dlu(b.S, b.T, b.V, b.W, [b.N], C, True)
        h0, _ = ox.x2c_direct(b.S, b.T, b.V, b.W, C, True)
        ok = np.abs(h - h0).max() <= 1e-13 * np.abs(h0).max()
        m = _mol(scale=0.0)
        h = _dlu(m, True)
        hf, _ = ox.x2c_direct(m.S, m.T, m.V, m.W, C, True)
        ok &= np.abs(h - hf).max() <= 1e-12 * np.abs(hf).max()
    except Exception:
        return False
    return bool(ok)


def _index_contiguous(off, N, Ntot, twocomp):
    # planted: atom spinors taken as one contiguous range
    n = 2 * N if twocomp else N
    return np.arange(2 * off, 2 * off + n) if twocomp else np.arange(off, off + n)


@pytest.mark.parametrize("name", ["contiguous_spinor_block", "us_without_r"])
def test_planted_dlu_mistakes_are_caught(name, monkeypatch):
    assert _pins_pass()
    if name == "contiguous_spinor_block":
        monkeypatch.setattr(ox, "atom_spinor_index", _index_contiguous)
    else:
        orig = ox.x2c_direct

        def direct_no_r(*a, **k):
            out = orig(*a, **k)
            if k.get("return_parts"):
                out[2]["R"] = np.eye(out[2]["R"].shape[0], dtype=out[2]["R"].dtype)   # planted: U^L = 1
            return out
        monkeypatch.setattr(ox, "x2c_direct", direct_no_r)
    assert not _pins_pass(), f"mutant {name} survived"


@pytest.mark.parametrize("twocomp", [False, True])
def test_dlu_pair_blocks_tile_the_molecular_h(twocomp):
    """The per-pair form (used for sampled checks at full size) reproduces
    every block of the molecular DLU h."""
    m = _mol()
    h, parts = ox.x2c_dlu(m.S, m.T, m.V, _W(m, twocomp), m.Ns, C, twocomp, return_parts=True)
    for A in range(len(BLOCKS)):
        for B in range(len(BLOCKS)):
            blk = ox.x2c_dlu_pair(m.T, m.V, _W(m, twocomp), m.Ns, A, B, parts, C, twocomp)
            ia = ox.atom_spinor_index(int(m.off[A]), int(m.Ns[A]), m.Ntot, twocomp)
            ib = ox.atom_spinor_index(int(m.off[B]), int(m.Ns[B]), m.Ntot, twocomp)
            assert np.abs(blk - h[np.ix_(ia, ib)]).max() <= 1e-13 * np.abs(h).max()
