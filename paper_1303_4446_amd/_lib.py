"""ctypes binding of libx2c (argument marshalling only).

Device memory and streams come from PyTorch; every step of the X2C build runs
in the HIP kernels of libx2c.so.  There is no CPU fallback: if the library is
missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libx2c.so")

SPINFREE, TWOCOMP = 1, 2
FP64, SPLIT_BF16, SPLIT_INT8 = 0, 1, 2
RED_QUATERNION, RED_COMPLEX = 0, 1
ROUTE_SIZE, ROUTE_DEVICE_WIDE, ROUTE_AUTO = 0, 1, 2

OK, EINVAL, EHIP, EBLOCK, ESCRATCH = 0, -1, -2, -3, -4
INFO_NAMES = {0: "ok", 1: "S not SPD", 2: "T not SPD", 3: "positive-energy subspace not resolved",
              4: "positive-energy branch size != n", 5: "renormalisation matrix not PD", 6: "non-finite input"}

EXPORTED = ("x2c_max_n", "x2c_device_wide_min_n", "x2c_workspace_bytes", "x2c_build", "x2c_build_batched", "x2c_build_batched_xr",
            "x2c_build_batched_noalloc", "x2c_bss_workspace_bytes", "x2c_bss_batched", "x2c_dkh_workspace_bytes",
            "x2c_dkh_batched", "x2c_dkh_products", "x2c_tuned_shape",
            "x2c_dlu_workspace_bytes", "x2c_dlu_assemble", "x2c_strerror", "x2c_release", "x2c_graph_enable",
            "x2c_stream_split", "x2c_autotune", "x2c_picture_change", "x2c_picture_change_kramers", "x2c_trace_enable", "x2c_trace_read",
            "x2c_trace_reset")


class X2CError(RuntimeError):
    def __init__(self, code: int, msg: str, info=None):
        super().__init__(f"{msg} (code {code})")
        self.code = code
        self.info = info


class _Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("prec", ctypes.c_int), ("ozaki_slices", ctypes.c_int),
                ("c", ctypes.c_double), ("reduction", ctypes.c_int), ("route", ctypes.c_int)]


_LIB = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libx2c.so (built in-tree by paper_1303_4446_amd.build)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} not built; run `python -m paper_1303_4446_amd.builder`")
    lib = ctypes.CDLL(p)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)
    optp = ctypes.POINTER(_Options)
    lib.x2c_max_n.argtypes = [i32]
    lib.x2c_max_n.restype = i32
    lib.x2c_device_wide_min_n.argtypes = [i32, i32]
    lib.x2c_device_wide_min_n.restype = i32
    lib.x2c_workspace_bytes.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int)]
    lib.x2c_workspace_bytes.restype = ctypes.c_size_t
    lib.x2c_build.argtypes = [optp, i32, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp,
                              ctypes.POINTER(ctypes.c_int)]
    lib.x2c_build.restype = i32
    lib.x2c_build_batched.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp,
                                      i64p, vp, i64p, vp, vp, vp, ctypes.c_size_t, vp]
    lib.x2c_build_batched.restype = i32
    lib.x2c_build_batched_noalloc.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp,
                                              i64p, vp, i64p, vp, vp, vp]
    lib.x2c_build_batched_noalloc.restype = i32
    lib.x2c_bss_workspace_bytes.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int)]
    lib.x2c_bss_workspace_bytes.restype = ctypes.c_size_t
    lib.x2c_bss_batched.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp, i64p, vp, i64p,
                                    vp, vp, vp, ctypes.c_size_t, vp]
    lib.x2c_bss_batched.restype = i32
    lib.x2c_dkh_workspace_bytes.argtypes = [optp, i32, i32, ctypes.POINTER(ctypes.c_int)]
    lib.x2c_dkh_workspace_bytes.restype = ctypes.c_size_t
    lib.x2c_dkh_batched.argtypes = [optp, i32, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp, i64p, vp,
                                    vp, vp, ctypes.c_size_t, vp]
    lib.x2c_dkh_batched.restype = i32
    lib.x2c_tuned_shape.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]
    lib.x2c_tuned_shape.restype = i32
    lib.x2c_dkh_products.argtypes = [i32]
    lib.x2c_dkh_products.restype = i32
    lib.x2c_build_batched_xr.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp,
                                         i64p, vp, i64p, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.x2c_build_batched_xr.restype = i32
    lib.x2c_dlu_workspace_bytes.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int)]
    lib.x2c_dlu_workspace_bytes.restype = ctypes.c_size_t
    lib.x2c_dlu_assemble.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), vp, vp, vp, i64p, vp, vp, vp,
                                     vp, ctypes.c_size_t, vp]
    lib.x2c_dlu_assemble.restype = i32
    lib.x2c_picture_change.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp, vp, vp, vp,
                                       vp, ctypes.c_size_t, vp]
    lib.x2c_picture_change.restype = i32
    lib.x2c_picture_change_kramers.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp, vp, vp, vp,
                                       vp, ctypes.c_size_t, vp]
    lib.x2c_picture_change_kramers.restype = i32
    lib.x2c_strerror.argtypes = [i32]
    lib.x2c_strerror.restype = ctypes.c_char_p
    lib.x2c_release.argtypes = []
    lib.x2c_release.restype = None
    lib.x2c_graph_enable.argtypes = [i32]
    lib.x2c_graph_enable.restype = i32
    lib.x2c_stream_split.argtypes = [i32]
    lib.x2c_stream_split.restype = i32
    lib.x2c_autotune.argtypes = [optp, i32, ctypes.POINTER(ctypes.c_int), i64p, vp, vp, vp, vp, i64p, vp, i64p, vp,
                                 vp, vp, ctypes.c_size_t, vp, i32, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int)]
    lib.x2c_autotune.restype = i32
    lib.x2c_trace_enable.argtypes = [i32]
    lib.x2c_trace_enable.restype = i32
    lib.x2c_trace_read.argtypes = [i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_longlong)]
    lib.x2c_trace_read.restype = i32
    lib.x2c_trace_reset.argtypes = []
    lib.x2c_trace_reset.restype = None
    if path is None:
        _LIB = lib
    return lib


def options(twocomp: bool, c: float, prec: int = FP64, slices: int = 0,
            reduction: int = RED_QUATERNION, route: int = 0) -> _Options:
    return _Options(TWOCOMP if twocomp else SPINFREE, prec, slices, float(c), reduction, route)


def strerror(code: int) -> str:
    return load().x2c_strerror(code).decode()


def max_n(twocomp: bool) -> int:
    return load().x2c_max_n(TWOCOMP if twocomp else SPINFREE)


def device_wide_min_n(twocomp: bool, n: int | None = None) -> int:
    """Smallest block size N that takes the device-wide path (whole-matrix
    products; no eigenvalues).  With n: set it (1 .. the
    batched limit + 1; 0 restores the default) and return the previous value;
    without: return the current value."""
    r = load().x2c_device_wide_min_n(TWOCOMP if twocomp else SPINFREE, -1 if n is None else int(n))
    if r < 0:
        raise X2CError(r, "invalid device-wide threshold")
    return int(r)


def workspace_bytes(Ns, twocomp: bool, c: float = 137.0, prec: int = FP64, route: int = 0,
                    reduction: int = RED_QUATERNION) -> int:
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    opt = options(twocomp, c, prec, 0, reduction, route)
    n = load().x2c_workspace_bytes(ctypes.byref(opt), len(Ns), Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if n == 0:
        raise X2CError(EINVAL, "invalid block sizes or options")
    return int(n)


def graph_enable(on: bool) -> bool:
    """Turn graph capture / replay of the build calls on or off; returns the
    previous setting."""
    return bool(load().x2c_graph_enable(1 if on else 0))


def stream_split(ways: int) -> int:
    """Run a batch as up to `ways` parts of about equal work on as many
    streams (1..4; 1 = the caller's stream only); returns the previous
    setting."""
    if ways not in (1, 2, 3, 4):
        raise ValueError("ways must be 1, 2, 3 or 4")
    return int(load().x2c_stream_split(int(ways)))


def trace_enable(on, level: int = 1) -> int:
    """Stage tracing on (level 1; level 2 adds per-launch matvec events) or
    off; returns the previous level."""
    return int(load().x2c_trace_enable(level if on else 0))


def trace_reset() -> None:
    load().x2c_trace_reset()


def trace_read() -> dict:
    """{stage: (total_ms, calls)} for the calls made while tracing was on."""
    lib = load()
    name = ctypes.c_char_p()
    ms = ctypes.c_double()
    cnt = ctypes.c_longlong()
    n = lib.x2c_trace_read(-1, None, None, None)
    out = {}
    for i in range(n):
        lib.x2c_trace_read(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt))
        out[name.value.decode()] = (ms.value, cnt.value)
    return out


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libx2c needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _dev(t, torch, dtype):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor of dtype %s" % dtype)
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class Batch:
    """Packed inputs of a batch on the device (layout of include/x2c.h)."""
    S: object
    T: object
    V: object
    W: object
    Ns: np.ndarray
    in_off: np.ndarray
    twocomp: bool

    @property
    def nblk(self) -> int:
        return len(self.Ns)

    def out_layout(self):
        n = self.Ns.astype(np.int64) * (2 if self.twocomp else 1)
        hsz = n * n * (2 if self.twocomp else 1)          # doubles
        h_off = np.zeros(self.nblk, dtype=np.int64)
        eps_off = np.zeros(self.nblk, dtype=np.int64)
        if self.nblk > 1:
            h_off[1:] = np.cumsum(hsz)[:-1]
            eps_off[1:] = np.cumsum(n)[:-1]
        return h_off, eps_off, int(hsz.sum()), int(n.sum())


def batch_to_device(packed: dict, twocomp: bool, device="cuda") -> Batch:
    torch = _torch()
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return Batch(f(packed["S"]), f(packed["T"]), f(packed["V"]), f(packed["W"]),
                 np.asarray(packed["Ns"], dtype=np.int32), np.asarray(packed["in_off"], dtype=np.int64), twocomp)


def build_batched_xr(batch: Batch, c: float, prec: int = FP64, slices: int = 0, workspace=None, stream=None,
                     reduction: int = RED_QUATERNION, route: int = 0):
    """Enqueue x2c_build_batched_xr.  Returns (h, eps, info, X, R) device
    tensors (X and R in the flat layout of h) and the workspace."""
    torch = _torch()
    lib = load()
    dev = batch.S.device
    h_off, eps_off, hsz, esz = batch.out_layout()
    h = torch.empty(hsz, dtype=torch.float64, device=dev)
    X = torch.empty(hsz, dtype=torch.float64, device=dev)
    R = torch.empty(hsz, dtype=torch.float64, device=dev)
    eps = torch.empty(esz, dtype=torch.float64, device=dev)
    info = torch.empty(batch.nblk, dtype=torch.int32, device=dev)
    wsb = workspace_bytes(batch.Ns, batch.twocomp, c, prec, route, reduction)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(batch.twocomp, c, prec, slices, reduction, route)
    Ns = np.ascontiguousarray(batch.Ns, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    in_off, ho, eo = i64(batch.in_off), i64(h_off), i64(eps_off)
    P = ctypes.POINTER(ctypes.c_int64)
    f64 = lambda t: _dev(t, torch, torch.float64)
    rc = lib.x2c_build_batched_xr(
        ctypes.byref(opt), batch.nblk, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), in_off.ctypes.data_as(P),
        f64(batch.S), f64(batch.T), f64(batch.V), f64(batch.W), ho.ctypes.data_as(P), f64(h),
        eo.ctypes.data_as(P), f64(eps), f64(X), f64(R), _dev(info, torch, torch.int32),
        ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return (h, eps, info, X, R), workspace


def picture_change(Ns, twocomp: bool, p_off, PLL, PSS, X, R, PLS=None, PSL=None, c: float = 137.0,
                   workspace=None, stream=None, out=None, time_even: bool = False):
    """Enqueue x2c_picture_change: per block P~ = R^H [P_LL + P_LS X +
    X^H P_SL + X^H P_SS X] R.  All matrices are flat device float64 tensors
    in the layout of h (block b at double offset p_off[b]); PLS / PSL may be
    None.  time_even (two-component only): x2c_picture_change_kramers, the
    quaternion products for operators of time-reversal form.  Returns (out,
    workspace)."""
    torch = _torch()
    lib = load()
    dev = PLL.device
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    po = np.ascontiguousarray(p_off, dtype=np.int64)
    if out is None:
        out = torch.empty_like(PLL)
    wsb = workspace_bytes(Ns, twocomp, c)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(twocomp, c)
    f64 = lambda t: None if t is None else _dev(t, torch, torch.float64)
    fn = lib.x2c_picture_change_kramers if time_even else lib.x2c_picture_change
    rc = fn(
        ctypes.byref(opt), len(Ns), Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        po.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), f64(PLL), f64(PLS), f64(PSL), f64(PSS), f64(X), f64(R),
        f64(out), ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return out, workspace


def dlu_workspace_bytes(Ns, twocomp: bool, c: float = 137.0) -> int:
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    opt = options(twocomp, c)
    n = load().x2c_dlu_workspace_bytes(ctypes.byref(opt), len(Ns), Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if n == 0:
        raise X2CError(EINVAL, "invalid atom sizes or options")
    return int(n)


def dlu_assemble(T, V, W, Ns, u_off, X, R, c: float, twocomp: bool, workspace=None, stream=None, H=None):
    """Enqueue x2c_dlu_assemble: molecular T, V (Ntot x Ntot) and W (Ntot x Ntot
    or 4 x Ntot x Ntot) device tensors, the atoms' X and R in the flat layout
    given by u_off (double offsets).  Returns (H, workspace); H is
    Ntot x Ntot float64 or 2Ntot x 2Ntot complex128."""
    torch = _torch()
    lib = load()
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    Ntot = int(Ns.sum())
    n = 2 * Ntot if twocomp else Ntot
    dev = T.device
    if H is None:
        H = torch.empty((n, n), dtype=torch.complex128 if twocomp else torch.float64, device=dev)
    wsb = dlu_workspace_bytes(Ns, twocomp, c)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(twocomp, c)
    uo = np.ascontiguousarray(u_off, dtype=np.int64)
    f64 = lambda t: _dev(t, torch, torch.float64)
    if not (H.is_cuda and H.is_contiguous() and H.numel() == n * n):
        raise ValueError("H must be a contiguous device tensor of the molecular size")
    rc = lib.x2c_dlu_assemble(ctypes.byref(opt), len(Ns), Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              f64(T), f64(V), f64(W), uo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              f64(X), f64(R), ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                              ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return H, workspace


def build_batched(batch: Batch, c: float, prec: int = FP64, slices: int = 0, workspace=None, out=None,
                  stream=None, reduction: int = RED_QUATERNION, route: int = 0):
    """Enqueue x2c_build_batched.  Returns (h_flat, eps_flat, info) device
    tensors (h_flat float64; complex blocks interleaved) and the workspace.
    route: ROUTE_SIZE (by block size), ROUTE_DEVICE_WIDE (every block on the
    device-wide path, eps NaN) or ROUTE_AUTO (the faster path for the whole
    batch when the eigenvalues are not needed; eps NaN where it took the
    device-wide path)."""
    torch = _torch()
    lib = load()
    dev = batch.S.device
    h_off, eps_off, hsz, esz = batch.out_layout()
    if out is None:
        h = torch.empty(hsz, dtype=torch.float64, device=dev)
        eps = torch.empty(esz, dtype=torch.float64, device=dev)
        info = torch.empty(batch.nblk, dtype=torch.int32, device=dev)
    else:
        h, eps, info = out
    wsb = workspace_bytes(batch.Ns, batch.twocomp, c, prec, route, reduction)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(batch.twocomp, c, prec, slices, reduction, route)
    Ns = np.ascontiguousarray(batch.Ns, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    in_off, ho, eo = i64(batch.in_off), i64(h_off), i64(eps_off)
    P = ctypes.POINTER(ctypes.c_int64)
    rc = lib.x2c_build_batched(
        ctypes.byref(opt), batch.nblk, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), in_off.ctypes.data_as(P),
        _dev(batch.S, torch, torch.float64), _dev(batch.T, torch, torch.float64),
        _dev(batch.V, torch, torch.float64), _dev(batch.W, torch, torch.float64),
        ho.ctypes.data_as(P), _dev(h, torch, torch.float64), eo.ctypes.data_as(P),
        _dev(eps, torch, torch.float64), _dev(info, torch, torch.int32),
        ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return (h, eps, info), workspace


def build_batched_noalloc(batch: Batch, c: float, prec: int = FP64, slices: int = 0, out=None, stream=None,
                          reduction: int = RED_QUATERNION):
    """Enqueue x2c_build_batched_noalloc (the library's static scratch instead
    of a workspace).  Returns (h_flat, eps_flat, info) device tensors; the
    output tensors are created here unless `out` is given."""
    torch = _torch()
    lib = load()
    dev = batch.S.device
    h_off, eps_off, hsz, esz = batch.out_layout()
    if out is None:
        out = (torch.empty(hsz, dtype=torch.float64, device=dev), torch.empty(esz, dtype=torch.float64, device=dev),
               torch.empty(batch.nblk, dtype=torch.int32, device=dev))
    h, eps, info = out
    opt = options(batch.twocomp, c, prec, slices, reduction)
    Ns = np.ascontiguousarray(batch.Ns, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    in_off, ho, eo = i64(batch.in_off), i64(h_off), i64(eps_off)
    P = ctypes.POINTER(ctypes.c_int64)
    rc = lib.x2c_build_batched_noalloc(
        ctypes.byref(opt), batch.nblk, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), in_off.ctypes.data_as(P),
        _dev(batch.S, torch, torch.float64), _dev(batch.T, torch, torch.float64),
        _dev(batch.V, torch, torch.float64), _dev(batch.W, torch, torch.float64),
        ho.ctypes.data_as(P), _dev(h, torch, torch.float64), eo.ctypes.data_as(P),
        _dev(eps, torch, torch.float64), _dev(info, torch, torch.int32), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return h, eps, info


def tuned_shape(Ns, twocomp: bool, c: float = 137.0, prec: int = FP64, slices: int = 0,
                reduction: int = RED_QUATERNION):
    """(found, ways, mv_res): the launch shape a batch of these block sizes
    would use, and whether it comes from x2c_autotune (this process or the
    cache file)."""
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    opt = options(twocomp, c, prec, slices, reduction)
    w, r = ctypes.c_int(0), ctypes.c_int(0)
    rc = load().x2c_tuned_shape(ctypes.byref(opt), len(Ns), Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                ctypes.byref(w), ctypes.byref(r))
    if rc < 0:
        raise X2CError(rc, strerror(rc))
    return bool(rc), w.value, r.value


def dkh_products(order: int) -> int:
    """2c matrix multiplications per block of x2c_dkh_batched at this order
    (-1 outside 1..14)."""
    return int(load().x2c_dkh_products(int(order)))


def bss_workspace_bytes(Ns, twocomp: bool, c: float = 137.0) -> int:
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    opt = options(twocomp, c)
    n = load().x2c_bss_workspace_bytes(ctypes.byref(opt), len(Ns), Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if n == 0:
        raise X2CError(EINVAL, "invalid block sizes or options")
    return int(n)


def dkh_workspace_bytes(Ns, twocomp: bool, order: int, c: float = 137.0) -> int:
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    opt = options(twocomp, c)
    n = load().x2c_dkh_workspace_bytes(ctypes.byref(opt), int(order), len(Ns),
                                       Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if n == 0:
        raise X2CError(EINVAL, "invalid block sizes, order or options")
    return int(n)


def bss_batched(batch: Batch, c: float, workspace=None, out=None, stream=None):
    """Enqueue x2c_bss_batched.  Returns ((h_flat, eps_flat, info), workspace)."""
    torch = _torch()
    lib = load()
    dev = batch.S.device
    h_off, eps_off, hsz, esz = batch.out_layout()
    if out is None:
        out = (torch.empty(hsz, dtype=torch.float64, device=dev), torch.empty(esz, dtype=torch.float64, device=dev),
               torch.empty(batch.nblk, dtype=torch.int32, device=dev))
    h, eps, info = out
    wsb = bss_workspace_bytes(batch.Ns, batch.twocomp, c)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(batch.twocomp, c)
    Ns = np.ascontiguousarray(batch.Ns, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    in_off, ho, eo = i64(batch.in_off), i64(h_off), i64(eps_off)
    P = ctypes.POINTER(ctypes.c_int64)
    f64 = lambda t: _dev(t, torch, torch.float64)
    rc = lib.x2c_bss_batched(
        ctypes.byref(opt), batch.nblk, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), in_off.ctypes.data_as(P),
        f64(batch.S), f64(batch.T), f64(batch.V), f64(batch.W), ho.ctypes.data_as(P), f64(h), eo.ctypes.data_as(P),
        f64(eps), _dev(info, torch, torch.int32), ctypes.c_void_p(workspace.data_ptr()),
        ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return out, workspace


def dkh_batched(batch: Batch, c: float, order: int, workspace=None, out=None, stream=None):
    """Enqueue x2c_dkh_batched.  Returns ((h_flat, info), workspace)."""
    torch = _torch()
    lib = load()
    dev = batch.S.device
    h_off, _, hsz, _ = batch.out_layout()
    if out is None:
        out = (torch.empty(hsz, dtype=torch.float64, device=dev), torch.empty(batch.nblk, dtype=torch.int32, device=dev))
    h, info = out
    wsb = dkh_workspace_bytes(batch.Ns, batch.twocomp, order, c)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(batch.twocomp, c)
    Ns = np.ascontiguousarray(batch.Ns, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    in_off, ho = i64(batch.in_off), i64(h_off)
    P = ctypes.POINTER(ctypes.c_int64)
    f64 = lambda t: _dev(t, torch, torch.float64)
    rc = lib.x2c_dkh_batched(
        ctypes.byref(opt), int(order), batch.nblk, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        in_off.ctypes.data_as(P), f64(batch.S), f64(batch.T), f64(batch.V), f64(batch.W), ho.ctypes.data_as(P),
        f64(h), _dev(info, torch, torch.int32), ctypes.c_void_p(workspace.data_ptr()),
        ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return out, workspace


def autotune(batch: Batch, c: float, prec: int = FP64, slices: int = 0, workspace=None, out=None, stream=None,
             reduction: int = RED_QUATERNION, reps: int = 3, route: int = 0):
    """x2c_autotune on the batch (writes the same outputs as build_batched).
    Returns (ways, mv_res) of the fastest launch shape, the outputs and the
    workspace."""
    torch = _torch()
    lib = load()
    dev = batch.S.device
    h_off, eps_off, hsz, esz = batch.out_layout()
    if out is None:
        out = (torch.empty(hsz, dtype=torch.float64, device=dev), torch.empty(esz, dtype=torch.float64, device=dev),
               torch.empty(batch.nblk, dtype=torch.int32, device=dev))
    h, eps, info = out
    wsb = workspace_bytes(batch.Ns, batch.twocomp, c, prec, route, reduction)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opt = options(batch.twocomp, c, prec, slices, reduction, route)
    Ns = np.ascontiguousarray(batch.Ns, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    in_off, ho, eo = i64(batch.in_off), i64(h_off), i64(eps_off)
    P = ctypes.POINTER(ctypes.c_int64)
    ways, res = ctypes.c_int(0), ctypes.c_int(0)
    rc = lib.x2c_autotune(
        ctypes.byref(opt), batch.nblk, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), in_off.ctypes.data_as(P),
        _dev(batch.S, torch, torch.float64), _dev(batch.T, torch, torch.float64),
        _dev(batch.V, torch, torch.float64), _dev(batch.W, torch, torch.float64),
        ho.ctypes.data_as(P), _dev(h, torch, torch.float64), eo.ctypes.data_as(P),
        _dev(eps, torch, torch.float64), _dev(info, torch, torch.int32),
        ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()), _stream_ptr(torch, stream),
        int(reps), ctypes.byref(ways), ctypes.byref(res))
    if rc != OK:
        raise X2CError(rc, strerror(rc))
    return (ways.value, res.value), out, workspace


def release() -> None:
    """x2c_release: drop cached plans, graphs, tuned launch shapes and trace events."""
    load().x2c_release()


def unpack_h(h_flat: np.ndarray, Ns, twocomp: bool):
    """Split a flat host copy of h into per-block matrices."""
    out = []
    o = 0
    for N in Ns:
        n = int(N) * (2 if twocomp else 1)
        if twocomp:
            blk = h_flat[o:o + 2 * n * n].view(np.complex128).reshape(n, n)
            o += 2 * n * n
        else:
            blk = h_flat[o:o + n * n].reshape(n, n)
            o += n * n
        out.append(blk)
    return out


def build(S, T, V, W, c: float, twocomp: bool, prec: int = FP64, slices: int = 0, workspace=None, stream=None,
          reduction: int = RED_QUATERNION, route: int = 0):
    """x2c_build on one block given as device tensors (S, T, V: N x N;
    W: N x N (spin-free) or 4 x N x N).  Returns (h, eps) device tensors.
    Raises X2CError with .info on a failed block."""
    torch = _torch()
    lib = load()
    N = int(S.shape[0])
    n = 2 * N if twocomp else N
    dev = S.device
    h = torch.empty((n, n), dtype=torch.complex128 if twocomp else torch.float64, device=dev)
    eps = torch.empty(n, dtype=torch.float64, device=dev)
    opt = options(twocomp, c, prec, slices, reduction, route)
    wsb = workspace_bytes([N], twocomp, c, prec, route, reduction)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    info = ctypes.c_int(0)
    rc = lib.x2c_build(ctypes.byref(opt), N, _dev(S, torch, torch.float64), _dev(T, torch, torch.float64),
                       _dev(V, torch, torch.float64), _dev(W, torch, torch.float64),
                       ctypes.c_void_p(h.data_ptr()), _dev(eps, torch, torch.float64),
                       ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()),
                       _stream_ptr(torch, stream), ctypes.byref(info))
    if rc != OK:
        raise X2CError(rc, strerror(rc) + (f": {INFO_NAMES.get(info.value)}" if rc == EBLOCK else ""),
                       info.value)
    return h, eps
