"""Per-block failure codes, forced from the host: a failed block reports its
info code and gets zero output, the other blocks of the batch are unaffected."""
import numpy as np
import pytest

from x2c_inputs import C_LIGHT, atom_block, neon_s20
from x2c_inputs.integrals import AtomBlock
from tests.test_gpu_parity import check_against_oracle, gpu_batched, _px

pytestmark = pytest.mark.gpu


def _mod(blk, **kw):
    d = dict(Z=blk.Z, S=blk.S.copy(), T=blk.T.copy(), V=blk.V.copy(), W=blk.W.copy())
    d.update(kw)
    return AtomBlock(**d)


def test_info_codes_in_one_batch():
    good = atom_block(8)
    sbad = good.S.copy(); sbad[3, 3] = -1.0
    tbad = good.T.copy(); tbad[2, 2] = -5.0
    vnan = good.V.copy(); vnan[1, 4] = np.nan; vnan[4, 1] = np.nan
    dup = neon_s20()                       # duplicated exponent: S and T singular
    Sd = dup.S.copy(); Td = dup.T.copy(); Vd = dup.V.copy(); Wd = dup.W.copy()
    for M in (Sd, Td, Vd, Wd[0]):
        M[1, :] = M[0, :]; M[:, 1] = M[:, 0]
    blocks = [good, _mod(good, S=sbad), _mod(good, T=tbad), _mod(good, V=vnan),
              AtomBlock(Z=10.0, S=Sd, T=Td, V=Vd, W=Wd), good]
    for twocomp in (False, True):
        hs, eps, info = gpu_batched(blocks, twocomp)
        assert list(info) == [0, 1, 2, 6, 1, 0], info
        for i in (1, 2, 3, 4):
            assert not np.any(hs[i]) and not np.any(eps[i])
        for i in (0, 5):
            W = good.W if twocomp else good.W[0]
            check_against_oracle(good.S, good.T, good.V, W, C_LIGHT, twocomp, hs[i], eps[i])


def test_branch_count_failure():
    """c = 1 with Z = 79: no clean split at -c^2 (info 4)."""
    blk = atom_block(79)
    hs, eps, info = gpu_batched([blk, atom_block(1)], False, c=1.0)
    assert info[0] == 4


def test_single_block_error_raises():
    px, torch = _px()
    blk = atom_block(6)
    S = blk.S.copy(); S[0, 0] = -1.0
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(px.X2CError) as ei:
        px.build(d(S), d(blk.T), d(blk.V), d(blk.W[0]), C_LIGHT, False)
    assert ei.value.code == px.EBLOCK and ei.value.info == 1
