#!/usr/bin/env python3
"""Benchmark: batched DLU X2C builds on one MI355X.

Default workload: the Ag309-like batch -- 309 two-component Z=47 atomic
blocks (s22 p18 d12 f8, N = 192 scalar functions, 384 spinors, 4c dimension
768), V and W^q of each block scaled by a seeded factor U(0.98, 1.02).

A step is one x2c_build_batched call over the whole batch with inputs already
resident in HBM.  W untimed warm-up steps, then K steps timed with HIP events
on the stream the library launches on (the library replays the call's
captured HIP graph).  A second, traced pass over K more steps (eager
launches with HIP events around every stage and every reduction-matvec
launch) gives the stage breakdown and the roofline of the dominant kernel.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "DLU X2C blocks/sec at fixed max|dE| vs FP64 oracle; split-prec vs plain FP64"

# MI355X peaks (AMD published figures)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def algorithmic_flops(stage: str, N: int, twocomp: bool) -> float | None:
    """Algorithmic real flops per block of a stage (complex multiply-add = 8
    flops; products with Hermitian output counted at half; diagonal scalings
    not counted)."""
    n = 2 * N if twocomp else N
    m = 2 * n
    cm = 4.0 if twocomp else 1.0          # complex vs real arithmetic
    if stage == "tridiag_4c":             # Householder tridiagonalisation: (4/3) m^3 mult-add pairs
        return cm * (4.0 / 3.0) * m ** 3
    if stage == "tridiag_Q":
        return cm * (4.0 / 3.0) * n ** 3
    if stage == "backtransform_4c":       # Q (m x m, m-1 reflectors) applied to m x n
        return cm * 2.0 * m * m * n
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
    block are counted (the 4c matrix and the renormalisation matrix)."""
    Ns = np.asarray(Ns, dtype=np.int64)
    if twocomp and reduction == "quaternion":
        dims = [(2 * Ns, 32), (Ns, 32)]
    elif twocomp:
        dims = [(4 * Ns, 16), (2 * Ns, 16)]
    else:
        dims = [(2 * Ns, 8), (Ns, 8)]
    total, launches = 0.0, 0
    for d, es in dims:
        maxd = int(d.max())
        if not twocomp and maxd <= 96:
            continue                      # single work-group reduction, no matvec launches
        launches += maxd - 1
        for dim in d:
            L = np.arange(int(dim) - 1, 0, -1, dtype=np.float64)   # len = dim - k - 1
            total += float(np.sum(L * (L + 1) / 2.0)) * es
    return total, launches


def recorded_traffic(kernel_src: str, summary: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel's source has changed
    since the counters were taken (or the summary is missing)."""
    import hashlib
    try:
        with open(os.path.join(HERE, summary)) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(("|", "#", "`")))
        with open(os.path.join(HERE, kernel_src), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
        if kv.get("source_sha256_16", "").strip() != h:
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
    return {"operator": "nuclear attraction (P_LL = V, P_SS = W/4c^2)", "ms_per_call": ms,
            "blocks_per_s": len(batch.Ns) / (ms / 1e3)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["ag309", "mixed512"], default="ag309")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--prec", choices=["fp64", "split", "split8"], default="fp64",
                    help="products of the X / L / S~ / R chain: FP64, bf16 slices, int8 slices")
    ap.add_argument("--reduction", choices=["quaternion", "complex"], default="quaternion",
                    help="two-component eigenproblem reduction")
    ap.add_argument("--check-blocks", type=int, default=3, help="blocks checked against the oracle")
    ap.add_argument("--cpu-blocks", type=int, default=12, help="blocks in the CPU oracle sample (0 = skip)")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--no-pct", action="store_true", help="skip the picture-change timing")
    ap.add_argument("--streams", type=int, choices=[1, 2, 3, 4], default=4,
                    help="run the batch as this many parts on as many streams")
    ap.add_argument("--no-graph", action="store_true", help="eager launches instead of graph replay")
    ap.add_argument("--autotune", action="store_true",
                    help="before the warm-up, let x2c_autotune pick the launch shape (streams, matvec residency)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the workload, copy a device buffer of this size once (a plain copy kernel "
                         "of known traffic for scaling hardware byte counters)")
    return ap.parse_args()


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


def accuracy_gate(blocks, hs, eps, twocomp, c, nsample, seed):
    """max|dE| (Eh) of the GPU h against the oracle's positive-energy 4c
    spectrum on a seeded sample of blocks, next to the oracle's own floor."""
    import oracle
    import oracle.routes as ox
    rng = np.random.default_rng(seed + 77)
    idx = rng.choice(len(blocks), size=min(nsample, len(blocks)), replace=False)
    dmax_b = dmax_a = floor_a = floor_b = 0.0
    for i in idx:
        b = blocks[int(i)]
        W = b.W if twocomp else b.W[0]
        e4 = oracle.dirac_positive_spectrum(b.S, b.T, b.V, W, c, twocomp)
        es = oracle.spectrum_of(hs[int(i)], b.S, twocomp)
        h0, _ = ox.x2c_direct(b.S, b.T, b.V, W, c, twocomp)
        e0 = oracle.spectrum_of(h0, b.S, twocomp)
        d = np.abs(es - e4)
        f = np.abs(e0 - e4)
        bd = e4 < 0
        dmax_a = max(dmax_a, float(d.max()))
        floor_a = max(floor_a, float(f.max()))
        if bd.any():
            dmax_b = max(dmax_b, float(d[bd].max()))
            floor_b = max(floor_b, float(f[bd].max()))
    return dict(max_dE_bound_Eh=dmax_b, max_dE_all_Eh=dmax_a, oracle_floor_bound_Eh=floor_b,
                oracle_floor_all_Eh=floor_a, checked_blocks=[int(i) for i in idx])


def cpu_baseline(blocks, twocomp, c, nblk_sample):
    """The oracle as it stands, timed on this host on a bounded sample."""
    import oracle.routes as ox
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    sample = blocks[:nblk_sample]
    t0 = time.perf_counter()
    for b in sample:
        ox.x2c_direct(b.S, b.T, b.V, b.W if twocomp else b.W[0], c, twocomp)
    dt = time.perf_counter() - t0
    return {"value": len(sample) / dt, "unit": "blocks/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {len(sample)} blocks of the same batch, sequential, x2c_direct with "
                      f"threaded LAPACK ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; --gpus must be 1 "
                                   "(the per-block DLU build shards over blocks: each GPU runs "
                                   "its own share of the batch with no communication)"}))
        sys.exit(2)
    import torch
    import paper_1303_4446_amd as px
    from x2c_inputs import C_LIGHT, pack_blocks

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    c = C_LIGHT
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr, flush=True)
        del src, dst
    blocks, twocomp, desc = workload(args.workload, args.seed)
    prec = {"fp64": px.FP64, "split": px.SPLIT_BF16, "split8": px.SPLIT_INT8}[args.prec]
    red = px.RED_QUATERNION if args.reduction == "quaternion" else px.RED_COMPLEX
    pk = pack_blocks(blocks, twocomp)
    batch = px.batch_to_device(pk, twocomp)
    if args.no_graph:
        px.graph_enable(False)
    px.stream_split(args.streams)
    stream = torch.cuda.current_stream()
    print(f"# workload: {desc}; prec {args.prec}", file=sys.stderr, flush=True)

    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned, out, ws = px.autotune(batch, c, prec=prec, stream=stream, reduction=red, reps=2)
        print(f"# autotune: {tuned[0]} streams, matvec {tuned[1]} work-groups per CU "
              f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    (h, eps, info), ws = px.build_batched(batch, c, prec=prec, stream=stream, reduction=red,
                                          workspace=ws if tuned else None)
    out = (h, eps, info)
    for _ in range(max(0, args.warmup - 1)):
        px.build_batched(batch, c, prec=prec, workspace=ws, out=out, stream=stream, reduction=red)
    torch.cuda.synchronize()
    print("# warm-up done", file=sys.stderr, flush=True)

    # timed region: the production path (graph replay of the whole call)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        px.build_batched(batch, c, prec=prec, workspace=ws, out=out, stream=stream, reduction=red)
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    print(f"# timed {args.steps} steps: {elapsed_ms:.1f} ms", file=sys.stderr, flush=True)

    # traced pass over the same steps (eager launches, HIP events on the call's
    # stream around every stage and every matvec launch).  A first traced
    # step, not recorded, fills the library's event pool, and the events are
    # collected after every step, so that no recorded step creates events
    # while its kernels run (event creation on the host would show up as gaps
    # inside the stage brackets).
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
        print(f"# traced pass done", file=sys.stderr, flush=True)

    info_h = info.cpu().numpy()
    if np.any(info_h != 0):
        raise SystemExit(f"blocks failed: {np.nonzero(info_h)[0][:10]} codes {info_h[info_h != 0][:10]}")
    hs = px.unpack_h(h.cpu().numpy(), batch.Ns, twocomp)

    nblk = len(blocks)
    ms_step = elapsed_ms / args.steps
    value = nblk * args.steps / (elapsed_ms / 1e3)

    acc = accuracy_gate(blocks, hs, eps, twocomp, c, args.check_blocks, args.seed)
    print(f"# accuracy {acc}", file=sys.stderr, flush=True)

    mv = stages.pop("k_tri_matvec", None)
    stage_ms = {k: v[0] / max(1, v[1]) for k, v in stages.items()}
    roofline = None
    if mv is not None and mv[1] > 0:
        total_b, launches = matvec_bytes(batch.Ns, twocomp, args.reduction)
        per_launch_b = total_b / max(1, launches)
        avg_ms = mv[0] / mv[1]
        achieved = per_launch_b / (avg_ms / 1e3) / 1e9
        traffic = None
        if args.workload == "ag309" and twocomp and args.reduction == "quaternion":
            traffic = recorded_traffic("paper_1303_4446_amd/csrc/k_matvec.hip",
                                       "profiles/k_tri_matvec_w_ag309_traffic.md")
        roofline = {"bound": "hbm", "kernel": "k_tri_matvec_w" if (twocomp and args.reduction == "quaternion")
                    else "k_tri_matvec", "achieved": achieved, "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                    "launch_us": avg_ms * 1e3, "bytes_per_launch": per_launch_b,
                    "launches_per_step": mv[1] / args.steps, "share_of_step": mv[0] / args.steps / ms_step}
    extra = {}
    for st in ("tridiag_4c", "backtransform_4c"):
        fl = [algorithmic_flops(st, int(N), twocomp) for N in batch.Ns]
        if None not in fl and st in stage_ms:
            extra[st + "_fp64_tflops"] = sum(fl) / (stage_ms[st] / 1e3) / 1e12
    chain = [st for st in CHAIN_STAGES if st in stage_ms]
    if twocomp and args.reduction == "quaternion" and args.prec == "fp64" and len(chain) == len(CHAIN_STAGES):
        n3 = float(np.sum(np.asarray(batch.Ns, dtype=np.float64) ** 3))
        ms = sum(stage_ms[st] for st in chain)
        extra["chain_fp64_tflops"] = CHAIN_FLOPS_PER_N3 * n3 / (ms / 1e3) / 1e12
        extra["chain_frac_of_fp64_peak"] = extra["chain_fp64_tflops"] / PEAK_FP64_TFLOPS

    pct = None if args.no_pct else time_picture_change(px, torch, batch, twocomp, c, prec, red, stream)
    cpu = cpu_baseline(blocks, twocomp, c, args.cpu_blocks) if args.cpu_blocks > 0 else None

    line = {
        "metric": METRIC, "value": value, "unit": "blocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "nblocks": nblk, "mode": "two-component" if twocomp else "spin-free",
                   "prec": args.prec, "reduction": args.reduction,
                   "streams": tuned[0] if tuned else args.streams,
                   "matvec_wg_per_cu": tuned[1] if tuned else 8, "autotuned": bool(tuned), **acc},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages_ms_per_step": {k: round(v, 4) for k, v in sorted(stage_ms.items(), key=lambda kv: -kv[1])},
        "stage_rates": extra,
        "picture_change": pct,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
