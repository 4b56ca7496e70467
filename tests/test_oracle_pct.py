"""Pins of the oracle's picture-change transformation (Sec. II: U^L and U^S
are kept for the picture change of property integrals; Eq. utrans with a
property's 4c matrix in place of D).

* The identity operator: its large-component matrix is S and its
  small-component matrix <sigma.p chi|sigma.p chi> = <p chi|.|p chi> = 2T
  (the cross-product part vanishes), so P_SS = 2T / 4c^2 = T / 2c^2 and the
  transformed operator is R^H S~ R, which the renormalisation makes equal to
  S (Eq. ulnonortho).  A dropped 1/4c^2, a reversed U^S = R X or a missing
  spin structure breaks it.
* The Dirac matrix itself (P_LL = V, P_LS = P_SL = T, P_SS = W/4c^2 - T,
  Eq. moddiraceq) gives back the Hamiltonian h of Eq. utrans.
"""
import numpy as np
import pytest

import oracle.routes as ox
from x2c_inputs import C_LIGHT as C, atom_block

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _parts(Z, twocomp):
    b = atom_block(Z)
    W = b.W if twocomp else b.W[0]
    h, _, parts = ox.x2c_direct(b.S, b.T, b.V, W, C, twocomp, return_parts=True)
    return b, h, parts


@pytest.mark.parametrize("twocomp", [False, True])
@pytest.mark.parametrize("Z", [6, 17])
def test_identity_operator_maps_to_the_metric(Z, twocomp):
    b, _, parts = _parts(Z, twocomp)
    N = b.S.shape[0]
    WO = np.stack([2.0 * b.T, np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))])
    P = ox.property_blocks(b.S, WO, C, twocomp)
    out = ox.picture_change(*P, parts["X"], parts["R"])
    Sx = ox.spin_blockdiag(b.S) if twocomp else b.S
    assert np.abs(out - Sx).max() <= 1e-11 * np.abs(Sx).max()


@pytest.mark.parametrize("twocomp", [False, True])
def test_dirac_matrix_gives_the_hamiltonian(twocomp):
    b, h, parts = _parts(8, twocomp)
    W = b.W if twocomp else b.W[0]
    Sx, Tx, Vx, Wx = ox.spinor_matrices(b.S, b.T, b.V, W, twocomp)
    out = ox.picture_change(Vx, Tx, Tx, Wx / (4.0 * C * C) - Tx, parts["X"], parts["R"])
    assert np.abs(out - h).max() <= 1e-12 * np.abs(h).max()


def test_multiplicative_operator_blocks_follow_eq_defw():
    """The small-component block of a multiplicative operator is W^O / 4c^2
    assembled like W (Eq. defw): alpha-alpha W0 + i Wz, alpha-beta Wy + i Wx."""
    rng = np.random.default_rng(3)
    N = 3
    O = rng.standard_normal((N, N))
    WO = rng.standard_normal((4, N, N))
    PLL, PLS, PSL, PSS = ox.property_blocks(O, WO, 2.0, True)
    assert np.allclose(PLL[:N, :N], O) and np.allclose(PLL[N:, N:], O) and not PLL[:N, N:].any()
    assert not PLS.any() and not PSL.any()
    assert np.allclose(PSS[:N, :N] * 16.0, WO[0] + 1j * WO[3])
    assert np.allclose(PSS[:N, N:] * 16.0, WO[2] + 1j * WO[1])
    assert np.allclose(PSS[N:, :N] * 16.0, -WO[2] + 1j * WO[1])
    assert np.allclose(PSS[N:, N:] * 16.0, WO[0] - 1j * WO[3])
