"""Host logic of the DKHn path (no GPU): the plan that x2c_dkh_batched runs
performs exactly the numbers of 2c matrix multiplications of Table I
(Sec. II, "The DKH approach", column "this work"), read from the golden
fixture."""
import os

import pytest

import paper_1303_4446_amd as px

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dkh_multiplications.txt")


def table_one():
    rows = [tuple(map(int, l.split())) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return dict(rows)


@pytest.mark.parametrize("order", range(2, 15))
def test_plan_multiplications_equal_table_one(order):
    assert px.dkh_products(order) == table_one()[order]


def test_plan_limits():
    assert px.dkh_products(1) == 0          # E_0 - c^2 + E_1: no product
    assert px.dkh_products(0) == -1 and px.dkh_products(15) == -1


def test_dkh_and_bss_workspace_queries():
    w2 = px.dkh_workspace_bytes([192], True, 2)
    w8 = px.dkh_workspace_bytes([192], True, 8)
    assert 0 < w2 < w8
    # DKH keeps no 4c buffers: far smaller than the X2C workspace of the block
    assert w8 < px.workspace_bytes([192], True)
    assert px.bss_workspace_bytes([192], True) > px.workspace_bytes([192], True)
    with pytest.raises(px.X2CError):
        px.dkh_workspace_bytes([192], True, 15)
