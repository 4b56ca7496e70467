"""The C ABI: library loads, exports what include/x2c.h declares, host-side
argument handling (CPU); argument validation through a real call (GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1303_4446_amd as px
from paper_1303_4446_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "x2c.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(x2c_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(_lib.EXPORTED)


def test_library_loads_and_exports_every_declared_symbol():
    lib = px.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_query_and_limits():
    lib = px.load()
    assert px.max_n(True) >= 192 and px.max_n(False) >= 200
    w1 = px.workspace_bytes([20], twocomp=False)
    w2 = px.workspace_bytes([20, 45], twocomp=False)
    w3 = px.workspace_bytes([192], twocomp=True)
    assert 0 < w1 < w2 and w3 > w2
    with pytest.raises(px.X2CError):
        px.workspace_bytes([0], twocomp=False)
    with pytest.raises(px.X2CError):
        px.workspace_bytes([px.max_n(True) + 1], twocomp=True)
    # invalid options -> 0
    opt = _lib.options(True, -1.0)
    N = (ctypes.c_int * 1)(10)
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) == 0
    opt = _lib._Options(7, 0, 0, 137.0, 0)
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) == 0
    opt = _lib.options(True, 137.0, prec=px.SPLIT_BF16, slices=9)   # beyond the slice limit
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) == 0
    opt = _lib.options(True, 137.0, prec=px.SPLIT_BF16, slices=8)
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) > 0
    opt = _lib.options(True, 137.0, prec=px.SPLIT_INT8)
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) > 0
    opt = _lib.options(True, 137.0, prec=3)             # unknown precision
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) == 0
    opt = _lib.options(True, 137.0, reduction=2)      # unknown reduction
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) == 0
    for red in (px.RED_QUATERNION, px.RED_COMPLEX):
        opt = _lib.options(True, 137.0, reduction=red)
        assert lib.x2c_workspace_bytes(ctypes.byref(opt), 1, N) > 0
    # empty batch needs no workspace
    opt = _lib.options(True, 137.0)
    assert lib.x2c_workspace_bytes(ctypes.byref(opt), 0, N) == 0


def test_strerror_covers_all_codes():
    for code in (0, -1, -2, -3, 1, 2, 3, 4, 5, 6):
        assert px.strerror(code) != "unknown code"
    assert px.strerror(99) == "unknown code"


def test_null_arguments_rejected_without_gpu_work():
    """Invalid arguments are caught on the host before any device call."""
    lib = px.load()
    opt = _lib.options(False, 137.0)
    info = ctypes.c_int(0)
    rc = lib.x2c_build(ctypes.byref(opt), 4, None, None, None, None, None, None, None, 0, None,
                       ctypes.byref(info))
    assert rc == px.EINVAL
    N = np.array([4], dtype=np.int32)
    off = np.zeros(1, dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    rc = lib.x2c_build_batched(ctypes.byref(opt), 1, N.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               off.ctypes.data_as(P), None, None, None, None, off.ctypes.data_as(P), None,
                               off.ctypes.data_as(P), None, None, None, 0, None)
    assert rc == px.EINVAL
    rc = lib.x2c_picture_change(ctypes.byref(opt), 1, N.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                off.ctypes.data_as(P), None, None, None, None, None, None, None, None, 0, None)
    assert rc == px.EINVAL
    rc = lib.x2c_autotune(ctypes.byref(opt), 1, N.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          off.ctypes.data_as(P), None, None, None, None, off.ctypes.data_as(P), None,
                          off.ctypes.data_as(P), None, None, None, 0, None, 3, None, None)
    assert rc == px.EINVAL
    # reps out of range is rejected before the batch is looked at
    fake = ctypes.c_void_p(16)
    rc = lib.x2c_autotune(ctypes.byref(opt), 1, N.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          off.ctypes.data_as(P), fake, fake, fake, fake, off.ctypes.data_as(P), fake,
                          off.ctypes.data_as(P), fake, fake, fake, 0, None, 0, None, None)
    assert rc == px.EINVAL
    # empty batch is a no-op
    rc = lib.x2c_build_batched(ctypes.byref(opt), 0, N.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               off.ctypes.data_as(P), None, None, None, None, off.ctypes.data_as(P), None,
                               off.ctypes.data_as(P), None, None, None, 0, None)
    assert rc == px.OK


@pytest.mark.gpu
def test_workspace_too_small_is_rejected():
    import torch
    from x2c_inputs import neon_s20
    blk = neon_s20()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    lib = px.load()
    opt = _lib.options(False, 137.0)
    h = torch.empty((20, 20), dtype=torch.float64, device="cuda")
    e = torch.empty(20, dtype=torch.float64, device="cuda")
    S, T, V, W = d(blk.S), d(blk.T), d(blk.V), d(blk.W[0])
    info = ctypes.c_int(0)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = lib.x2c_build(ctypes.byref(opt), 20, vp(S), vp(T), vp(V), vp(W), vp(h), vp(e), vp(small), 1024,
                       None, ctypes.byref(info))
    assert rc == px.EINVAL


def test_device_wide_threshold_and_workspace():
    """Size classes: blocks above the batched limit take the device-wide path
    (up to x2c_max_n); the threshold can be lowered, never raised."""
    assert px.device_wide_min_n(True) == 257 and px.device_wide_min_n(False) == 513
    assert px.max_n(True) == 4096 and px.max_n(False) == 8192
    w_batched = px.workspace_bytes([192], twocomp=True)
    old = px.device_wide_min_n(True, 100)
    try:
        assert old == 257
        assert px.device_wide_min_n(True) == 100
        assert px.workspace_bytes([192], twocomp=True) != w_batched
        assert px.workspace_bytes([99], twocomp=True) == px.workspace_bytes([99], twocomp=True)
    finally:
        px.device_wide_min_n(True, 0)
    assert px.device_wide_min_n(True) == 257
    assert px.workspace_bytes([192], twocomp=True) == w_batched
    with pytest.raises(px.X2CError):
        px.device_wide_min_n(True, 258)
    # the full 13-atom silver molecule (N = 2496): one GPU's HBM holds it easily
    w = px.workspace_bytes([2496], twocomp=True)
    assert 1e9 < w < 24e9
    # routes: every block device-wide, or the faster path for the whole batch
    # (device-wide for a few silver blocks, batched for 309 of them)
    w_dw = px.workspace_bytes([192], twocomp=True, route=px.ROUTE_DEVICE_WIDE)
    assert w_dw != w_batched
    with pytest.raises(px.X2CError):
        px.workspace_bytes([192], twocomp=True, route=3)
    # the automatic route's workspace covers either path (whichever a later
    # x2c_autotune measures faster)
    for Ns in ([192], [192] * 13, [192] * 309, [24, 123, 200]):
        w_auto = px.workspace_bytes(Ns, twocomp=True, route=px.ROUTE_AUTO)
        assert w_auto == max(px.workspace_bytes(Ns, twocomp=True),
                             px.workspace_bytes(Ns, twocomp=True, route=px.ROUTE_DEVICE_WIDE))
    # BSS, DKHn and the allocation-free entry stay on the batched path
    with pytest.raises(px.X2CError):
        px.bss_workspace_bytes([300], twocomp=True)
    with pytest.raises(px.X2CError):
        px.dkh_workspace_bytes([300], twocomp=True, order=2)
