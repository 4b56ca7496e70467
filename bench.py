#!/usr/bin/env python3
"""Benchmark: batched DLU X2C builds on one MI355X.

Default workload: the Ag309-like batch -- 309 two-component Z=47 atomic
blocks (s22 p18 d12 f8, N = 192 scalar functions, 384 spinors, 4c dimension
768), V and W^q of each block scaled by a seeded factor U(0.98, 1.02).

A step is one x2c_build_batched call over the whole batch with inputs already
resident in HBM.  W untimed warm-up steps, then K steps timed with HIP events
on the stream the library launches on (the library replays the call's
captured HIP graph); `value` is the FP64 product chain.  The same run then
times the split-precision products (bf16 and int8 slices) on the same batch,
and scores all three against the FP64 oracle on a seeded sample of blocks.
A traced pass (eager launches with HIP events around every stage and every
reduction-matvec launch) gives the stage breakdown and the roofline of the
dominant kernel.  The CPU oracle is timed first, before anything touches the
GPU.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "DLU X2C blocks/sec at fixed max|dE| vs FP64 oracle; split-prec vs plain FP64"

# MI355X peaks (AMD published figures)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# bound-state accuracy target per eigenvalue (Eh)
DE_TARGET = 1e-8

# The paper's own timings of the X2C step (context, not targets): serial CPU
# runs of the whole one-electron Hamiltonian evaluation in its program,
# molecular DLU assembly included.
PAPER_TIMINGS = [
    {"what": "X2C, two-component (spin-orbit), DLU, Ag13 C1 (13 atomic blocks, 119 primitives per atom)",
     "seconds": 21.0, "blocks_per_s": 13 / 21.0, "hardware": "Intel Xeon E5430, one core",
     "source": "Table tab_cputime12c"},
    {"what": "X2C, two-component (spin-orbit), full (no local approximation), Ag13 C1",
     "seconds": 1707.5, "hardware": "Intel Xeon E5430, one core", "source": "Table tab_cputime12c"},
    {"what": "X2C_loc, two-component (SO), Ag13 C1", "seconds": 20.0, "blocks_per_s": 13 / 20.0,
     "hardware": "Intel Xeon X3460 2.8 GHz", "source": "Table tab:res4"},
    {"what": "X2C_loc, scalar-relativistic, Ag309 Oh (309 atomic blocks)", "seconds": 1875.0,
     "blocks_per_s": 309 / 1875.0, "hardware": "Intel Xeon X3460 2.8 GHz", "source": "Table tab:res4"},
    {"what": "DKH2 / DKH3 / DKH4 / DKH8 / BSS, two-component (SO), DLU, Ag13 C1",
     "seconds": {"dkh2": 13.2, "dkh3": 14.0, "dkh4": 15.3, "dkh8": 27.3, "bss": 21.6},
     "hardware": "Intel Xeon E5430, one core", "source": "Table tab_cputime12c"},
]


def algorithmic_flops(stage: str, N: int, twocomp: bool, reduction: str = "quaternion") -> float | None:
    """Algorithmic real flops per block of a stage, counted for the arithmetic
    the path actually does: a real multiply-add is 2 flops, a complex one 8,
    a quaternion one 32.  Householder tridiagonalisation of a dimension-d
    Hermitian matrix: (2/3) d^3 multiply-adds of the scalar type; applying the
    d - 1 reflectors to a d x r block: d^2 r multiply-adds.  The
    two-component quaternion reductions act on the d = 2N quaternion form of
    the 4c matrix (d = N for the renormalisation matrix); the complex
    reduction on the complex 4N / 2N forms; spin-free on real 2N / N."""
    if twocomp and reduction == "quaternion":
        d4, dq, rhs, fl = 2 * N, N, N, 32.0
    elif twocomp:
        d4, dq, rhs, fl = 4 * N, 2 * N, 2 * N, 8.0
    else:
        d4, dq, rhs, fl = 2 * N, N, N, 2.0
    if stage == "tridiag_4c":
        return fl * (2.0 / 3.0) * d4 ** 3
    if stage == "tridiag_Q":
        return fl * (2.0 / 3.0) * dq ** 3
    if stage == "backtransform_4c":
        return fl * d4 * d4 * rhs
    return None


# The product chain after X~ (quaternion form, FP64): stages and their
# algorithmic real flops per block in units of N^3 (N quaternion rows).  A
# quaternion multiply-add is 16 real multiply-adds (32 flops), a real scalar
# matrix times a quaternion 4 (8 flops); Hermitian outputs and triangular
# real factors count half.  chain_SL: T X (8), W'' X (32), X^H (W'' X) (16);
# chain_Q: X~^H X~ (16); chain_R: two triangular factors (4 + 4); chain_h:
# L R (32), R^H (L R) (16).
CHAIN_STAGES = ("chain_SL", "chain_Q", "chain_R", "chain_h")
CHAIN_FLOPS_PER_N3 = 8 + 32 + 16 + 16 + 8 + 32 + 16


def matvec_bytes(Ns, twocomp: bool, reduction: str) -> tuple[float, int]:
    """Algorithmic HBM bytes of all tridiagonal-reduction matvec launches of
    one step, and the number of launches.  Unit: one element of the lower
    triangle (diagonal included) of the trailing Hermitian matrix read once
    per column step; a launch covers every block at that step.  Element
    sizes: quaternion 32 B, complex 16 B, real 8 B.  Both reductions of a
    block are counted (the 4c matrix and the renormalisation matrix).  A
    quaternion reduction stops its matvec launches at the unblocked tail
    (quaternion_tail_start), whose columns one kernel per block reduces."""
    Ns = np.asarray(Ns, dtype=np.int64)
    quatred = twocomp and reduction == "quaternion"
    if quatred:
        dims = [(2 * Ns, 32), (Ns, 32)]
    elif twocomp:
        dims = [(4 * Ns, 16), (2 * Ns, 16)]
    else:
        dims = [(2 * Ns, 8), (Ns, 8)]
    ncols = (lambda n: min(n - 1, quaternion_tail_start(n))) if quatred else (lambda n: n - 1)
    total, launches = 0.0, 0
    for d, es in dims:
        maxd = int(d.max())
        if not twocomp and maxd <= 96:
            continue                      # single work-group reduction, no matvec launches
        launches += ncols(maxd)
        for dim in d:
            L = int(dim) - 1 - np.arange(ncols(int(dim)), dtype=np.float64)   # len = dim - k - 1
            total += float(np.sum(L * (L + 1) / 2.0)) * es
    return total, launches


def quaternion_tail_start(n: int, tail_max: int = 64, panel: int = 16) -> int:
    """First column of the unblocked tail of a quaternion reduction of
    dimension n: the first panel boundary at or after n - 1 - tail_max."""
    s = n - 1 - tail_max
    return 0 if s <= 0 else -(-s // panel) * panel


# the dominant kernel's source and the headers whose code it inlines
MATVEC_SOURCES = ("paper_1303_4446_amd/csrc/k_matvec.hip", "paper_1303_4446_amd/csrc/x2c_device.h",
                  "paper_1303_4446_amd/csrc/x2c_tridiag.h")


def sources_hash(kernel_srcs) -> str:
    """First 16 hex digits of the SHA-256 of the files' bytes, in order."""
    import hashlib
    srcs = (kernel_srcs,) if isinstance(kernel_srcs, str) else tuple(kernel_srcs)
    h = hashlib.sha256()
    for src in srcs:
        with open(os.path.join(HERE, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel_srcs, summary: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel's sources (the file
    and the headers it inlines) have changed since the counters were taken
    (or the summary is missing)."""
    try:
        with open(os.path.join(HERE, summary)) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(("|", "#", "`")))
        if kv.get("source_sha256_16", "").strip() != sources_hash(kernel_srcs):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def time_picture_change(px, torch, batch, twocomp, c, prec, red, stream, calls=3):
    """Throughput of x2c_picture_change over the whole batch for the nuclear
    attraction as the property (P_LL = V, P_SS = W / 4c^2 in the form of
    Eq. defw, P_LS = P_SL = 0), with the batch's own X and R.  The property
    matrices are assembled on the device from the batch's V and W."""
    (_, _, info, X, R), ws = px.build_batched_xr(batch, c, prec=prec, stream=stream, reduction=red)
    h_off, _, hsz, _ = batch.out_layout()
    PLL = torch.zeros(hsz, dtype=torch.float64, device="cuda")
    PSS = torch.zeros(hsz, dtype=torch.float64, device="cuda")
    q4 = 1.0 / (4.0 * c * c)
    for b, N in enumerate(batch.Ns):
        N = int(N)
        o, io = int(h_off[b]), int(batch.in_off[b])
        V = batch.V[io:io + N * N].view(N, N)
        if twocomp:
            W = batch.W[4 * io:4 * io + 4 * N * N].view(4, N, N)
            n = 2 * N
            L = PLL[o:o + 2 * n * n].view(n, n, 2)
            L[:N, :N, 0] = V
            L[N:, N:, 0] = V
            P = PSS[o:o + 2 * n * n].view(n, n, 2)
            P[:N, :N, 0], P[:N, :N, 1] = q4 * W[0], q4 * W[3]
            P[:N, N:, 0], P[:N, N:, 1] = q4 * W[2], q4 * W[1]
            P[N:, :N, 0], P[N:, :N, 1] = -q4 * W[2], q4 * W[1]
            P[N:, N:, 0], P[N:, N:, 1] = q4 * W[0], -q4 * W[3]
        else:
            PLL[o:o + N * N] = batch.V[io:io + N * N]
            PSS[o:o + N * N] = q4 * batch.W[io:io + N * N]
    out, ws = px.picture_change(batch.Ns, twocomp, h_off, PLL, PSS, X, R, c=c, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        px.picture_change(batch.Ns, twocomp, h_off, PLL, PSS, X, R, c=c, workspace=ws, stream=stream, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    if not bool(torch.isfinite(out).all()) or bool((info != 0).any()):
        return None
    res = {"operator": "nuclear attraction (P_LL = V, P_SS = W/4c^2)", "ms_per_call": ms,
           "blocks_per_s": len(batch.Ns) / (ms / 1e3)}
    if twocomp:
        # the operator is time-even: the quaternion products of
        # x2c_picture_change_kramers, checked against the complex products
        outq, _ = px.picture_change(batch.Ns, True, h_off, PLL, PSS, X, R, c=c, workspace=ws, stream=stream,
                                    time_even=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(calls):
            px.picture_change(batch.Ns, True, h_off, PLL, PSS, X, R, c=c, workspace=ws, stream=stream, out=outq,
                              time_even=True)
        e1.record(stream)
        torch.cuda.synchronize()
        msq = e0.elapsed_time(e1) / calls
        dev = float((outq - out).abs().max() / out.abs().max())
        res["time_even_quaternion"] = {"ms_per_call": msq, "blocks_per_s": len(batch.Ns) / (msq / 1e3),
                                       "max_rel_diff_vs_complex": dev}
    return res


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["ag309", "mixed512"], default="ag309")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--prec", choices=["fp64", "split", "split8"], default="fp64",
                    help="products of the X / L / S~ / R chain of the headline figure: FP64, bf16 slices, "
                         "int8 slices")
    ap.add_argument("--split-steps", type=int, default=5,
                    help="timed steps of each split-precision comparison run (0 = skip the comparison)")
    ap.add_argument("--fw-steps", type=int, default=5,
                    help="timed steps of each BSS / DKHn run on the same batch (0 = skip)")
    ap.add_argument("--dkh-orders", default="2,3,4,8", help="DKH orders timed in the BSS / DKHn comparison")
    ap.add_argument("--reduction", choices=["quaternion", "complex"], default="quaternion",
                    help="two-component eigenproblem reduction")
    ap.add_argument("--check-blocks", type=int, default=3, help="blocks checked against the oracle")
    ap.add_argument("--cpu-blocks", type=int, default=2,
                    help="blocks per core in each timed run of the CPU oracle sample (0 = skip)")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--no-pct", action="store_true", help="skip the picture-change timing")
    ap.add_argument("--streams", type=int, choices=[1, 2, 3, 4], default=4,
                    help="run the batch as this many parts on as many streams")
    ap.add_argument("--no-graph", action="store_true", help="eager launches instead of graph replay")
    ap.add_argument("--autotune", action="store_true",
                    help="before the warm-up, let x2c_autotune pick the launch shape (streams, matvec residency)")
    ap.add_argument("--full-steps", type=int, default=2,
                    help="timed full (non-local) builds of the 13-atom silver molecule against its DLU "
                         "approximation (0 = skip)")
    ap.add_argument("--full-precs", default="fp64,bf16", help="product-chain arithmetic of the full builds")
    ap.add_argument("--only-full", action="store_true",
                    help="run only the full-versus-DLU comparison (a profiling aid: prints its JSON object)")
    ap.add_argument("--no-full-spectra", action="store_true",
                    help="skip the CPU eigensolves that score the full and DLU spectra")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the workload, copy a device buffer of this size once (a plain copy kernel "
                         "of known traffic for scaling hardware byte counters)")
    return ap.parse_args(argv)


def workload(name: str, seed: int):
    from x2c_inputs.configs import ag309_dlu, mixed_dlu
    if name == "ag309":
        blocks = ag309_dlu(seed)
        desc = (f"ag309_dlu: 309 two-component Z=47 blocks (s22 p18 d12 f8, N=192, 384 spinors, 4c dim 768), "
                f"V,W scaled U(0.98,1.02), seed {seed}")
        return blocks, True, desc
    blocks = mixed_dlu(seed, 512)
    desc = f"mixed_dlu: 512 two-component blocks, Z uniform in {{1,6,8,17,29,47,79}}, seed {seed}"
    return blocks, True, desc


# ---------------------------------------------------------------------------
# accuracy against the FP64 oracle
# ---------------------------------------------------------------------------

def oracle_references(blocks, twocomp, c, idx):
    """Per sampled block: the oracle's positive 4c spectrum (brute force),
    the spectrum of the oracle's own X2C h with metric S, and its eps."""
    import oracle
    import oracle.routes as ox
    refs = {}
    for i in idx:
        b = blocks[int(i)]
        W = b.W if twocomp else b.W[0]
        e4 = oracle.dirac_positive_spectrum(b.S, b.T, b.V, W, c, twocomp)
        h0, e0 = ox.x2c_direct(b.S, b.T, b.V, W, c, twocomp)
        refs[int(i)] = dict(e4=e4, ex=oracle.spectrum_of(h0, b.S, twocomp), eps=e0)
    return refs


def score(blocks, twocomp, refs, hs, eps_blocks):
    """max|dE| (Eh) of the GPU h (eigenvalues of h with metric S, Eq. 2ceoeq)
    per eigenvalue against (a) the oracle's X2C spectrum and (b) the positive
    4c spectrum, over bound states (E < 0) and over all states; the oracle's
    own distance to the 4c spectrum (its floor); and the GPU's returned eps
    against the oracle's.  `pass` = bound-state max|dE| <= 1e-8 Eh against
    both references."""
    import oracle
    r = dict(max_dE_bound_vs_oracle_Eh=0.0, max_dE_all_vs_oracle_Eh=0.0, max_dE_bound_Eh=0.0,
             max_dE_all_Eh=0.0, oracle_floor_bound_Eh=0.0, oracle_floor_all_Eh=0.0, max_deps_rel=0.0)
    for i, ref in refs.items():
        es = oracle.spectrum_of(hs[i], blocks[i].S, twocomp)
        bd = ref["e4"] < 0
        dx = np.abs(es - ref["ex"])
        d4 = np.abs(es - ref["e4"])
        fl = np.abs(ref["ex"] - ref["e4"])
        r["max_dE_all_vs_oracle_Eh"] = max(r["max_dE_all_vs_oracle_Eh"], float(dx.max()))
        r["max_dE_all_Eh"] = max(r["max_dE_all_Eh"], float(d4.max()))
        r["oracle_floor_all_Eh"] = max(r["oracle_floor_all_Eh"], float(fl.max()))
        if bd.any():
            r["max_dE_bound_vs_oracle_Eh"] = max(r["max_dE_bound_vs_oracle_Eh"], float(dx[bd].max()))
            r["max_dE_bound_Eh"] = max(r["max_dE_bound_Eh"], float(d4[bd].max()))
            r["oracle_floor_bound_Eh"] = max(r["oracle_floor_bound_Eh"], float(fl[bd].max()))
        r["max_deps_rel"] = max(r["max_deps_rel"], float(np.abs(eps_blocks[i] - ref["eps"]).max()
                                                          / np.abs(ref["eps"]).max()))
    r["pass"] = bool(r["max_dE_bound_vs_oracle_Eh"] <= DE_TARGET and r["max_dE_bound_Eh"] <= DE_TARGET)
    r["checked_blocks"] = sorted(refs)
    return r


def split_eps(eps_flat, Ns, twocomp):
    n = np.asarray(Ns, dtype=np.int64) * (2 if twocomp else 1)
    offs = np.concatenate([[0], np.cumsum(n)])
    return [eps_flat[offs[i]:offs[i + 1]] for i in range(len(Ns))]


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on this host
# ---------------------------------------------------------------------------

def _oracle_time(job):
    """Worker: time x2c_direct on a few blocks with one BLAS thread."""
    blocks, twocomp, c = job
    import oracle.routes as ox
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for b in blocks:
            ox.x2c_direct(b.S, b.T, b.V, b.W if twocomp else b.W[0], c, twocomp)
        return time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(blocks, twocomp, c, per_core, runs=3):
    """The oracle's x2c_direct timed on this host's cores, median of `runs`:
    (i) one core (one BLAS thread), `per_core` blocks per run; (ii) a pool of
    worker processes, one BLAS thread each, `per_core` blocks per worker per
    run.  The pool is capped at 16 workers (this host's share of CPUs on a
    shared GPU node) and is forked before the GPU is initialised."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    workers = max(1, min(ncpu, 16))
    single = [_oracle_time((blocks[:per_core], twocomp, c)) for _ in range(runs)]
    t1 = statistics.median(single)
    jobs = [(blocks[(w * per_core) % len(blocks):(w * per_core) % len(blocks) + per_core], twocomp, c)
            for w in range(workers)]
    ctx = mp.get_context("fork")
    pool_t = []
    with ctx.Pool(workers) as pool:
        for _ in range(runs):
            t0 = time.perf_counter()
            pool.map(_oracle_time, jobs, chunksize=1)
            pool_t.append(time.perf_counter() - t0)
    tp = statistics.median(pool_t)
    nb_pool = sum(len(j[0]) for j in jobs)
    return {"value": nb_pool / tp, "unit": "blocks/s", "cores": workers, "kind": "oracle",
            "sample": (f"x2c_direct on the first blocks of the same batch, {per_core} per worker, "
                       f"{workers} worker processes with one BLAS thread each, median of {runs} runs "
                       f"({tp:.1f} s per run)"),
            "single_core_blocks_per_s": per_core / t1, "single_core_s_per_block": t1 / per_core,
            "host_cpus": ncpu, "cpu_model": cpu_model(), "runs_s": {"single": single, "pool": pool_t}}


# ---------------------------------------------------------------------------

def copy_rate_gbps(torch, mib: int = 1024, reps: int = 5) -> float:
    """Bytes moved (read + written) per second by a plain device-to-device
    copy of a mib-MiB buffer, median of reps copies timed with events: the
    HBM rate this part reaches in practice, beside the published peak."""
    n = (mib << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (float(np.median(ms)) / 1e3) / 1e9


def time_steps(px, torch, batch, c, prec, red, stream, ws, out, steps):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        px.build_batched(batch, c, prec=prec, workspace=ws, out=out, stream=stream, reduction=red)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def time_fw(px, torch, batch, c, stream, steps, method, order=0):
    """Blocks/s of x2c_bss_batched or x2c_dkh_batched on the batch (graph
    replay, same launch as the X2C timing) and the host copy of h."""
    run = (lambda ws=None, out=None: px.bss_batched(batch, c, workspace=ws, out=out, stream=stream)) \
        if method == "bss" else \
        (lambda ws=None, out=None: px.dkh_batched(batch, c, order, workspace=ws, out=out, stream=stream))
    out, ws = run()
    run(ws, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        run(ws, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    info = out[-1].cpu().numpy()
    hs = px.unpack_h(out[0].cpu().numpy(), batch.Ns, batch.twocomp)
    del ws, out
    return ms, hs, info


def score_fw(blocks, twocomp, c, refs, hs, method, order):
    """Bound-state max|dE| of eig(h, S) against the positive 4c spectrum (the
    method's own error for DKHn, exact decoupling for BSS) on the sampled
    blocks, and h against the oracle on the first of them."""
    import oracle
    import oracle.fw as ofw
    r = {"max_dE_bound_vs_4c_Eh": 0.0}
    for i, ref in refs.items():
        es = oracle.spectrum_of(hs[i], blocks[i].S, twocomp)
        bd = ref["e4"] < 0
        r["max_dE_bound_vs_4c_Eh"] = max(r["max_dE_bound_vs_4c_Eh"], float(np.abs(es - ref["e4"])[bd].max()))
    if refs:
        i = min(refs)
        b = blocks[i]
        W = b.W if twocomp else b.W[0]
        h0 = ofw.bss(b.S, b.T, b.V, W, c, twocomp)[0] if method == "bss" else \
            ofw.dkh(b.S, b.T, b.V, W, c, twocomp, order)
        r["h_rel_err_vs_oracle"] = float(np.abs(hs[i] - h0).max() / np.abs(h0).max())
        r["oracle_block"] = i
    return r


def full_vs_dlu(px, torch, c, stream, steps, precs, spectra=True):
    """The full (non-local) two-component X2C of the 13-atom silver molecule
    (N = 2496, 4992 spinors, 4c dimension 9984; one block on the device-wide
    path) against its DLU approximation (13 atomic blocks on the batched
    path, then the molecular assembly of Eqs. dlutrans, r2ctransatom, utrans),
    both timed on the GPU with the inputs resident.  Accuracy against values
    the oracle wrote (tests/golden/ag13_full_seed0.npz: rows of h and h V for
    a seeded V, the positive 4c eigenvalues): the full h is exact decoupling,
    so its bound states match the 4c ones; the DLU h carries the local
    approximation's error."""
    import scipy.linalg as sla
    from x2c_inputs import pack_blocks
    from x2c_inputs.configs import ag13_molecule
    mol = ag13_molecule(0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    S, T, V, W = d(mol.S), d(mol.T), d(mol.V), d(mol.W)
    gold = os.path.join(HERE, "tests", "golden", "ag13_full_seed0.npz")
    ref = np.load(gold) if os.path.exists(gold) else None
    S2 = None
    nb = None
    if ref is not None:
        e4 = ref["e4"]
        nb = int((e4 < 0).sum())

    def bound_de(h):
        nonlocal S2
        if ref is None or not spectra:
            return None
        if S2 is None:
            S2 = np.zeros((2 * mol.Ntot, 2 * mol.Ntot))
            S2[:mol.Ntot, :mol.Ntot] = mol.S
            S2[mol.Ntot:, mol.Ntot:] = mol.S
        es = sla.eigh(0.5 * (h + h.conj().T), S2, eigvals_only=True, subset_by_index=[0, nb - 1])
        return float(np.abs(es - e4[:nb]).max())

    def probe_err(h):
        if ref is None:
            return None
        return float(max(np.abs(h @ ref["V"] - ref["probes"]).max() / np.abs(ref["probes"]).max(),
                         np.abs(h[ref["row_index"]] - ref["rows"]).max() / float(ref["hmax"])))

    res = {"workload": f"ag13_molecule(0): 13 coupled two-component Z=47 blocks, N={mol.Ntot}, "
                       f"{2 * mol.Ntot} spinors, 4c dimension {4 * mol.Ntot} complex, coupling scale {mol.scale:g}",
           "bound_states": nb, "steps": steps}
    ws = torch.empty(px.workspace_bytes([mol.Ntot], True, c), dtype=torch.uint8, device="cuda")
    names = {"fp64": px.FP64, "bf16": px.SPLIT_BF16, "int8": px.SPLIT_INT8}
    full = {}
    for name in precs:
        p = names[name]
        h, _ = px.build(S, T, V, W, c, True, prec=p, workspace=ws, stream=stream)   # warm-up
        ts = []
        for _ in range(steps):
            t0 = time.perf_counter()
            h, eps = px.build(S, T, V, W, c, True, prec=p, workspace=ws, stream=stream)   # synchronises
            ts.append((time.perf_counter() - t0) * 1e3)
        hc = h.cpu().numpy()
        full[name] = {"ms": statistics.median(ts), "h_rel_err_vs_oracle": probe_err(hc),
                      "bound_dE_max": bound_de(hc), "eps_nan": bool(torch.isnan(eps).all().item())}
        print(f"# full {name}: {full[name]}", file=sys.stderr, flush=True)
        del h, hc
    # traced pass of the FP64 build: stage times and the Newton-Schulz step
    # counts; the sign iteration's products against the FP64 matrix-core peak
    if "fp64" in full:
        px.trace_reset()
        px.trace_enable(True, level=1)
        px.build(S, T, V, W, c, True, workspace=ws, stream=stream)
        tr = px.trace_read()
        px.trace_enable(False)
        px.trace_reset()
        st = {k: round(v[0], 3) for k, v in tr.items() if not k.endswith("_steps")}
        steps_ns = {k[:-6]: int(v[1]) for k, v in tr.items() if k.endswith("_steps")}
        n4, nh = 2 * mol.Ntot, mol.Ntot      # quaternion dimensions: 4c matrix, h
        # one quaternion multiply-add = 32 real flops; a Hermitian product
        # forms the lower triangle, n^2 (n + 1) / 2 multiply-adds
        herm = lambda n: 32.0 * n * n * (n + 1) / 2
        # sign: two Hermitian products per step; x_solve: the coupled
        # iteration on P_LL (three per step) and X~ = (P_SL Z) Z (two general)
        fl = {"sign_4c": steps_ns.get("sign_4c", 0) * 2 * herm(n4),
              "x_solve": steps_ns.get("x_solve", 0) * 3 * herm(nh) + 2 * 32.0 * nh ** 3}
        rates = {k: fl[k] / (st[k] / 1e3) / 1e12 for k in fl if st.get(k)}
        full["fp64"].update({"stages_ms": st, "newton_schulz_steps": steps_ns,
                             "stage_fp64_tflops": {k: round(v, 2) for k, v in rates.items()}})
        if "sign_4c" in rates:
            full["fp64"]["roofline"] = {"bound": "mfma", "kernel": "k_gemm_q_mfma (sign iteration products)",
                                        "achieved": rates["sign_4c"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                        "frac": rates["sign_4c"] / PEAK_FP64_TFLOPS,
                                        "flops": fl["sign_4c"], "stage_ms": st["sign_4c"]}
        print(f"# full fp64 traced: {st} steps {steps_ns} rates {rates}", file=sys.stderr, flush=True)
    del ws
    res["full"] = full
    # DLU: the atomic blocks (X and R kept) and the assembly; the atomic
    # blocks by size (batched path, eigenvalues written), and by the faster
    # path for this batch (thirteen blocks: device-wide, no eigenvalues)
    atoms = [mol.atom(A) for A in range(len(mol.Ns))]
    bt = px.batch_to_device(pack_blocks(atoms, True), True)
    h_off = bt.out_layout()[0]
    for key, route in (("dlu", px.ROUTE_SIZE), ("dlu_auto_route", px.ROUTE_AUTO)):
        (hb, eb, info, X, R), wsb = px.build_batched_xr(bt, c, stream=stream, route=route)
        H, wsa = px.dlu_assemble(T, V, W, mol.Ns, h_off, X, R, c, True, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            (hb, eb, info, X, R), wsb = px.build_batched_xr(bt, c, workspace=wsb, stream=stream, route=route)
            H, wsa = px.dlu_assemble(T, V, W, mol.Ns, h_off, X, R, c, True, workspace=wsa, stream=stream, H=H)
        e1.record(stream)
        torch.cuda.synchronize()
        Hc = H.cpu().numpy()
        res[key] = {"ms": e0.elapsed_time(e1) / steps, "blocks_ok": bool((info.cpu().numpy() == 0).all()),
                    "atomic_blocks_device_wide": bool(torch.isnan(eb).all().item()),
                    "h_rel_err_vs_full_oracle": probe_err(Hc), "bound_dE_max": bound_de(Hc)}
        print(f"# {key}: {res[key]}", file=sys.stderr, flush=True)
        del wsb, wsa, X, R, hb, eb, H
    if "fp64" in full:
        res["full_over_dlu_time"] = full["fp64"]["ms"] / res["dlu"]["ms"]
    return res


def host_outputs(px, out, batch, twocomp):
    h, eps, info = out
    info_h = info.cpu().numpy().copy()
    hs = px.unpack_h(h.cpu().numpy().copy(), batch.Ns, twocomp)
    return hs, split_eps(eps.cpu().numpy().copy(), batch.Ns, twocomp), info_h


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; --gpus must be 1 "
                                   "(the per-block DLU build shards over blocks: each GPU runs "
                                   "its own share of the batch with no communication)"}))
        sys.exit(2)
    c_light = __import__("x2c_inputs").C_LIGHT
    if args.only_full:
        import torch
        import paper_1303_4446_amd as px
        precs = [p for p in args.full_precs.split(",") if p]
        res = full_vs_dlu(px, torch, c_light, torch.cuda.current_stream(), max(1, args.full_steps), precs,
                          spectra=not args.no_full_spectra)
        print(json.dumps({"full_vs_dlu": res}), flush=True)
        return
    blocks, twocomp, desc = workload(args.workload, args.seed)

    # CPU baseline first: its worker processes are forked before the GPU is initialised
    cpu = None
    if args.cpu_blocks > 0:
        cpu = cpu_baseline(blocks, twocomp, c_light, args.cpu_blocks)
        print(f"# cpu baseline: {cpu['value']:.2f} blocks/s on {cpu['cores']} cores "
              f"({cpu['single_core_s_per_block']:.2f} s per block on one core)", file=sys.stderr, flush=True)

    import torch
    import paper_1303_4446_amd as px
    from x2c_inputs import pack_blocks

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    c = c_light
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr, flush=True)
        del src, dst
    precs = {"fp64": px.FP64, "split": px.SPLIT_BF16, "split8": px.SPLIT_INT8}
    prec = precs[args.prec]
    red = px.RED_QUATERNION if args.reduction == "quaternion" else px.RED_COMPLEX
    pk = pack_blocks(blocks, twocomp)
    batch = px.batch_to_device(pk, twocomp)
    if args.no_graph:
        px.graph_enable(False)
    px.stream_split(args.streams)
    stream = torch.cuda.current_stream()
    print(f"# workload: {desc}; prec {args.prec}", file=sys.stderr, flush=True)

    tuned = None
    ws = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned, _, ws = px.autotune(batch, c, prec=prec, stream=stream, reduction=red, reps=2)
        print(f"# autotune: {tuned[0]} streams, matvec {tuned[1]} work-groups per CU "
              f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    out, ws = px.build_batched(batch, c, prec=prec, stream=stream, reduction=red, workspace=ws)
    for _ in range(max(0, args.warmup - 1)):
        px.build_batched(batch, c, prec=prec, workspace=ws, out=out, stream=stream, reduction=red)
    torch.cuda.synchronize()
    print("# warm-up done", file=sys.stderr, flush=True)

    # timed region: the production path (graph replay of the whole call)
    elapsed_ms = time_steps(px, torch, batch, c, prec, red, stream, ws, out, args.steps)
    print(f"# timed {args.steps} steps: {elapsed_ms:.1f} ms", file=sys.stderr, flush=True)
    # the outputs of the timed replays are the ones scored
    hs, eps_b, info_h = host_outputs(px, out, batch, twocomp)
    if np.any(info_h != 0):
        raise SystemExit(f"blocks failed: {np.nonzero(info_h)[0][:10]} codes {info_h[info_h != 0][:10]}")
    nblk = len(blocks)
    ms_step = elapsed_ms / args.steps
    value = nblk * args.steps / (elapsed_ms / 1e3)

    # split-precision products vs the plain FP64 chain, same batch and launch
    split_runs = {}
    if args.split_steps > 0:
        for name in ("bf16", "int8"):
            p = px.SPLIT_BF16 if name == "bf16" else px.SPLIT_INT8
            if p == prec:
                continue
            so, _ = px.build_batched(batch, c, prec=p, workspace=ws, stream=stream, reduction=red)
            torch.cuda.synchronize()
            ms = time_steps(px, torch, batch, c, p, red, stream, ws, so, args.split_steps)
            shs, seps, sinfo = host_outputs(px, so, batch, twocomp)
            split_runs[name] = dict(ms=ms / args.split_steps, hs=shs, eps=seps, info=sinfo)
            print(f"# split {name}: {ms / args.split_steps:.1f} ms per step", file=sys.stderr, flush=True)
            del so

    # BSS and DKHn on the same batch (free-particle FW based decouplings)
    fw_runs = {}
    if args.fw_steps > 0 and args.prec == "fp64" and args.reduction == "quaternion":
        for method, order in [("bss", 0)] + [("dkh", int(o)) for o in args.dkh_orders.split(",") if o]:
            name = "bss" if method == "bss" else f"dkh{order}"
            ms, fhs, finfo = time_fw(px, torch, batch, c, stream, args.fw_steps, method, order)
            fw_runs[name] = dict(ms=ms, hs=fhs, info=finfo, method=method, order=order)
            print(f"# {name}: {ms:.1f} ms per step", file=sys.stderr, flush=True)

    # traced pass over the same steps (eager launches, HIP events on the call's
    # stream around every stage and every matvec launch).  A first traced
    # step, not recorded, fills the library's event pool, and the events are
    # collected after every step, so that no recorded step creates events
    # while its kernels run.
    stages = {}
    if not args.no_trace:
        px.trace_reset()
        px.trace_enable(True, level=2)
        px.build_batched(batch, c, prec=prec, workspace=ws, out=out, stream=stream, reduction=red)
        torch.cuda.synchronize()
        px.trace_reset()
        for _ in range(args.steps):
            px.build_batched(batch, c, prec=prec, workspace=ws, out=out, stream=stream, reduction=red)
            torch.cuda.synchronize()
            for k, (ms, cnt) in px.trace_read().items():
                a = stages.get(k, (0.0, 0))
                stages[k] = (a[0] + ms, a[1] + cnt)
            px.trace_reset()
        px.trace_enable(False)
        print("# traced pass done", file=sys.stderr, flush=True)

    rng = np.random.default_rng(args.seed + 77)
    idx = rng.choice(nblk, size=min(args.check_blocks, nblk), replace=False) if args.check_blocks > 0 else []
    refs = oracle_references(blocks, twocomp, c, idx)
    acc = score(blocks, twocomp, refs, hs, eps_b) if refs else {}
    print(f"# accuracy {acc}", file=sys.stderr, flush=True)
    split = None
    if split_runs:
        split = {"fp64": {"blocks_per_s": value, "ms_per_step": ms_step,
                          **{k: v for k, v in acc.items() if k != "checked_blocks"}}}
        for name, r in split_runs.items():
            ok = bool(np.all(r["info"] == 0))
            sc = score(blocks, twocomp, refs, r["hs"], r["eps"]) if (refs and ok) else {}
            split[name] = {"blocks_per_s": nblk / (r["ms"] / 1e3), "ms_per_step": r["ms"],
                           "slices": 7 if name == "bf16" else 8, "steps": args.split_steps, "blocks_ok": ok,
                           **{k: v for k, v in sc.items() if k != "checked_blocks"}}
            split[name]["faster_than_fp64"] = bool(r["ms"] < ms_step)
        print(f"# split {json.dumps(split)}", file=sys.stderr, flush=True)

    fwres = None
    if fw_runs:
        fwres = {}
        for name, r in fw_runs.items():
            ok = bool(np.all(r["info"] == 0))
            d = {"blocks_per_s": nblk / (r["ms"] / 1e3), "ms_per_step": r["ms"], "steps": args.fw_steps,
                 "blocks_ok": ok}
            if r["method"] == "dkh":
                d["products_per_block"] = px.dkh_products(r["order"])
            if ok:
                d.update(score_fw(blocks, twocomp, c, refs, r["hs"], r["method"], r["order"]))
            fwres[name] = d
        print(f"# fw {json.dumps(fwres)}", file=sys.stderr, flush=True)

    mv = stages.pop("k_tri_matvec", None)
    stage_ms = {k: v[0] / max(1, v[1]) for k, v in stages.items()}
    roofline = None
    if mv is not None and mv[1] > 0:
        total_b, launches = matvec_bytes(batch.Ns, twocomp, args.reduction)
        per_launch_b = total_b / max(1, launches)
        if abs(mv[1] / args.steps - launches) > 0.5:
            # the byte model's column schedule no longer matches the library's
            print(f"# warning: {mv[1] / args.steps:.0f} matvec launches per step traced, "
                  f"{launches} in the byte model", file=sys.stderr, flush=True)
        avg_ms = mv[0] / mv[1]
        achieved = per_launch_b / (avg_ms / 1e3) / 1e9
        traffic = None
        if args.workload == "ag309" and twocomp and args.reduction == "quaternion":
            traffic = recorded_traffic(MATVEC_SOURCES,
                                       "profiles/k_tri_matvec_w_ag309_traffic.md")
        copy_gbs = copy_rate_gbps(torch)
        roofline = {"bound": "hbm", "kernel": "k_tri_matvec_w" if (twocomp and args.reduction == "quaternion")
                    else "k_tri_matvec", "achieved": achieved, "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                    "launch_us": avg_ms * 1e3, "bytes_per_launch": per_launch_b,
                    "launches_per_step": mv[1] / args.steps, "share_of_step": mv[0] / args.steps / ms_step,
                    # the memory level the operands come from: the measured HBM traffic per
                    # launch over the launch time, against a plain 1 GiB copy of this run
                    "copy_GBps": copy_gbs,
                    "traffic_GBps": None if traffic is None else traffic / (avg_ms / 1e3) / 1e9,
                    "traffic_frac_of_copy": None if traffic is None else traffic / (avg_ms / 1e3) / 1e9 / copy_gbs}
    extra = {}
    for st in ("tridiag_4c", "tridiag_Q", "backtransform_4c"):
        fl = [algorithmic_flops(st, int(N), twocomp, args.reduction) for N in batch.Ns]
        if None not in fl and st in stage_ms:
            extra[st + "_fp64_tflops"] = sum(fl) / (stage_ms[st] / 1e3) / 1e12
    chain = [st for st in CHAIN_STAGES if st in stage_ms]
    if twocomp and args.reduction == "quaternion" and args.prec == "fp64" and len(chain) == len(CHAIN_STAGES):
        n3 = float(np.sum(np.asarray(batch.Ns, dtype=np.float64) ** 3))
        ms = sum(stage_ms[st] for st in chain)
        extra["chain_fp64_tflops"] = CHAIN_FLOPS_PER_N3 * n3 / (ms / 1e3) / 1e12
        extra["chain_frac_of_fp64_peak"] = extra["chain_fp64_tflops"] / PEAK_FP64_TFLOPS

    pct = None if args.no_pct else time_picture_change(px, torch, batch, twocomp, c, prec, red, stream)
    fvd = None
    if args.full_steps > 0:
        del out, ws
        torch.cuda.empty_cache()
        precs = [p for p in args.full_precs.split(",") if p]
        fvd = full_vs_dlu(px, torch, c, stream, args.full_steps, precs, spectra=not args.no_full_spectra)

    line = {
        "metric": METRIC, "value": value, "unit": "blocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.prec == "fp64" else "f64 (split products)",
        "data": "synthetic",
        "config": {"workload": desc, "nblocks": nblk, "mode": "two-component" if twocomp else "spin-free",
                   "prec": args.prec, "reduction": args.reduction,
                   "streams": tuned[0] if tuned else args.streams,
                   "matvec_wg_per_cu": tuned[1] if tuned else 8, "autotuned": bool(tuned)},
        "accuracy": acc,
        "split": split,
        "bss_dkh": fwres,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_timings": PAPER_TIMINGS,
        "stages_ms_per_step": {k: round(v, 4) for k, v in sorted(stage_ms.items(), key=lambda kv: -kv[1])},
        "stage_rates": extra,
        "picture_change": pct,
        "full_vs_dlu": fvd,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
