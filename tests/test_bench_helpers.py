"""Host-side helpers of bench.py: algorithmic byte counts of the reduction
matvec, the counter-profile reader and the chain flop count (no GPU)."""
import hashlib
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def brute_matvec_bytes(Ns, dim_of, es, skip_small, tail=False):
    """Column by column: the matvec at step k reads the lower triangle
    (diagonal included) of the trailing (d - k - 1)-square matrix.  With
    tail: the steps stop at the first multiple of 16 that leaves at most 64
    columns to reduce."""
    def steps(d):
        if not tail:
            return d - 1
        k = 0
        while d - 1 - k > 64:
            k += 16
        return min(k, d - 1)
    total, launches = 0.0, 0
    dims = [dim_of(int(N)) for N in Ns]
    if skip_small and max(dims) <= 96:
        return 0.0, 0
    launches = steps(max(dims))
    for d in dims:
        for k in range(steps(d)):
            L = d - k - 1
            total += L * (L + 1) // 2 * es
    return total, launches


@pytest.mark.parametrize("Ns", [[5], [7, 3, 12], [40, 40], [33, 70, 41], [192, 100]])
def test_matvec_bytes_quaternion_matches_column_count(Ns):
    tot, nl = bench.matvec_bytes(Ns, True, "quaternion")
    b4, l4 = brute_matvec_bytes(Ns, lambda N: 2 * N, 32, False, tail=True)
    bq, lq = brute_matvec_bytes(Ns, lambda N: N, 32, False, tail=True)
    assert nl == l4 + lq
    assert tot == pytest.approx(b4 + bq, rel=0, abs=0)


def test_matvec_bytes_complex_and_real():
    Ns = [30, 50]
    tot, nl = bench.matvec_bytes(Ns, True, "complex")
    b4, l4 = brute_matvec_bytes(Ns, lambda N: 4 * N, 16, False)
    bq, lq = brute_matvec_bytes(Ns, lambda N: 2 * N, 16, False)
    assert (tot, nl) == (b4 + bq, l4 + lq)
    # spin-free: reductions of dimension <= 96 use the one-work-group kernel
    tot, nl = bench.matvec_bytes([20, 40], False, "complex")
    assert (tot, nl) == (0.0, 0)
    tot, nl = bench.matvec_bytes([60], False, "complex")
    b4, l4 = brute_matvec_bytes([60], lambda N: 2 * N, 8, True)
    assert (tot, nl) == (b4, l4)


def test_ag309_bytes_per_launch():
    tot, nl = bench.matvec_bytes([192] * 309, True, "quaternion")
    assert nl == 320 + 128          # the last 63 and 63 columns: the unblocked tail
    assert tot / nl == pytest.approx(2.323984e8, rel=1e-6)


def test_chain_flops_unit():
    # 5 quaternion products (2 full at 32 N^3 flops, 3 Hermitian at 16) and 3
    # real-factor products (T X full at 8, two triangular at 4) after X~
    assert bench.CHAIN_FLOPS_PER_N3 == 2 * 32 + 3 * 16 + 8 + 2 * 4


def test_recorded_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source")
    h = hashlib.sha256(b"kernel source").hexdigest()[:16]
    prof = tmp_path / "p.md"
    prof.write_text(f"# title\n\n| a | b |\n\nsource: k.hip\nsource_sha256_16: {h}\ntraffic_bytes_per_launch: 1.5e+08\n")
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    assert bench.recorded_traffic("k.hip", "p.md") == 1.5e8
    src.write_bytes(b"kernel source, changed")
    assert bench.recorded_traffic("k.hip", "p.md") is None
    assert bench.recorded_traffic("k.hip", "missing.md") is None
    # several sources: an edit of an inlined header invalidates the figure too
    hdr = tmp_path / "k.h"
    hdr.write_bytes(b"header")
    src.write_bytes(b"kernel source")
    h2 = hashlib.sha256(b"kernel source" + b"header").hexdigest()[:16]
    prof.write_text(f"source: k.hip, k.h\nsource_sha256_16: {h2}\ntraffic_bytes_per_launch: 2.5e+08\n")
    assert bench.recorded_traffic(("k.hip", "k.h"), "p.md") == 2.5e8
    hdr.write_bytes(b"header, changed")
    assert bench.recorded_traffic(("k.hip", "k.h"), "p.md") is None


def test_committed_profile_is_readable():
    """The committed counter summary carries a source hash and a traffic
    figure; the benchmark reports the figure only while the hash matches
    the kernel source (None after an edit, until the counters are retaken)."""
    path = os.path.join(ROOT, "profiles", "k_tri_matvec_w_ag309_traffic.md")
    with open(path) as f:
        kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(("|", "#", "`")))
    assert len(kv["source_sha256_16"].strip()) == 16
    t = float(kv["traffic_bytes_per_launch"])
    assert 1.0e8 < t < 1.0e9
    v = bench.recorded_traffic(bench.MATVEC_SOURCES, "profiles/k_tri_matvec_w_ag309_traffic.md")
    assert v is None or v == t


@pytest.mark.parametrize("stage", ["tridiag_4c", "tridiag_Q", "backtransform_4c"])
def test_quaternion_stage_flops_are_half_the_complex_ones(stage):
    """The quaternion reductions do half the real arithmetic of the complex
    reductions of the same two-component block; the complex counts are the
    standard ones ((16/3) d^3 for a complex Hermitian tridiagonalisation of
    dimension d, 8 d^2 r for applying its reflectors to d x r)."""
    N = 192
    q = bench.algorithmic_flops(stage, N, True, "quaternion")
    cx = bench.algorithmic_flops(stage, N, True, "complex")
    assert q == pytest.approx(cx / 2, rel=1e-15)
    m, n = 4 * N, 2 * N
    ref = {"tridiag_4c": 16 / 3 * m ** 3, "tridiag_Q": 16 / 3 * n ** 3, "backtransform_4c": 8 * m * m * n}[stage]
    assert cx == pytest.approx(ref, rel=1e-15)
    # spin-free: real symmetric (4/3) d^3 and 2 d^2 r
    sf = bench.algorithmic_flops(stage, N, False)
    ref_sf = {"tridiag_4c": 4 / 3 * (2 * N) ** 3, "tridiag_Q": 4 / 3 * N ** 3,
              "backtransform_4c": 2 * (2 * N) ** 2 * N}[stage]
    assert sf == pytest.approx(ref_sf, rel=1e-15)


def test_score_reports_both_references_and_pass_flag():
    """score(): per-eigenvalue distances of the spectrum of a given h against
    the oracle's X2C spectrum and the 4c spectrum, with the pass flag at
    1e-8 Eh on bound states."""
    import oracle
    from x2c_inputs import C_LIGHT, atom_block
    import oracle.routes as ox
    blk = atom_block(6)
    refs = bench.oracle_references([blk], False, C_LIGHT, [0])
    h0, e0 = ox.x2c_direct(blk.S, blk.T, blk.V, blk.W[0], C_LIGHT, False)
    r = bench.score([blk], False, refs, [h0], [e0])
    assert r["pass"] and r["max_dE_bound_vs_oracle_Eh"] < 1e-10 and r["max_deps_rel"] == 0.0
    hb = h0 + 1e-6 * blk.S                    # every eigenvalue moves up by 1e-6 Eh
    r = bench.score([blk], False, refs, [hb], [e0])
    assert not r["pass"]
    assert r["max_dE_bound_vs_oracle_Eh"] == pytest.approx(1e-6, rel=1e-3)
    assert oracle.spectrum_of(hb, blk.S, False)[0] > refs[0]["ex"][0]
