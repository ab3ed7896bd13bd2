"""Throughput of the LC covariance path on one MI355X.

One step = the whole path on device-resident int32 catalogues of the
1000-mock, 1e5-galaxy workload: chaining-mesh build, DD/DR/RR pair counts of
every task, split Landy-Szalay xi + multipoles (float64), and the float32-MFMA
covariances with the float64 linear construction and its Cholesky/eigenvalue
check.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config c2]
                    [--no-cpu] [--no-per-mock] [--no-autotune]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-tests/s and LC-covariance mocks/hour at 1 GPU, batched vs per-mock"
# Integer-ALU roofline: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one 32/64-bit
# lane-op per lane per clock for add/compare/24-bit multiply and float64 FMA).
PEAK_OPS = 256 * 64 * 2.4e9
# Algorithmic work per binned pair (a pair within r_max): exact squared
# distance and range test (~14 ops), exact r and mu bin (~20 ops), one
# histogram increment.
OPS_PER_BINNED_PAIR = 35
# Pair tests the CPU baseline runs at most (about 10-30 s on 8-16 host cores).
CPU_SAMPLE_TESTS = 3.0e10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(src: str) -> str:
    """C++ source with comments and blank space removed (string literals in
    these files hold no comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash() -> str:
    """sha256[:16] of the pair-count kernel's code and of the mesh build
    whose layout it reads (paircount.hip, lc_internal.hpp and cells.hip,
    comments and layout removed, so that only a change to the code
    invalidates the measured traffic)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("paircount.hip", "lc_internal.hpp", "cells.hip"):
        with open(os.path.join(ROOT, "paper_2205_11852_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(config: str, n_mock: int, wl_mocks: int):
    """HBM bytes per launch of the pair-count kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (copy-calibrated), or None when
    the summary is missing, was taken on another workload, or the kernel
    source has changed since the counters were read."""
    path = os.path.join(ROOT, "profiles", "k_pair_count_%s_traffic.md" % config)
    if n_mock != wl_mocks or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source") != kernel_source_hash() or "traffic_bytes_per_launch" not in kv:
        return None
    return int(kv["traffic_bytes_per_launch"])


def workload_text(wl, n_mock: int) -> str:
    """What a workload is, with its sizes."""
    if wl.geometry == "periodic":
        where = "%g Mpc/h periodic box" % wl.box_mpc
    elif wl.geometry == "wedge":
        where = "open 60x60 deg wedge, comoving distance 1200-2400 Mpc/h, n(chi) falling 3x"
    else:
        where = "open 1500x1500x300 Mpc/h slab"
    if wl.per_mock_randoms:
        rnd = "two random sub-catalogues of each mock's size"
    else:
        rnd = "shared pool of %d x %d randoms" % (wl.n_subsets, wl.subset_size)
    los = {"z": "z line of sight", "mid": "midpoint line of sight",
           "rppi": "(r_p, pi) along z"}[wl.los]
    return ("%s: %d mocks x Poisson(%g) clustered galaxies, %s, %s, %d r-bins to %g Mpc/h x %d mu-bins, %s"
            % (wl.name, n_mock, wl.n_mean, where, rnd, wl.n_r, wl.r_max_mpc, wl.n_mu, los))


def paper_slab(args, torch, lc, stream) -> dict:
    """The paper's own workload shape (Sect. 4.1, 4.3, 5.3): clustered slabs of
    156 158 points on average in an open 1500 x 1500 x 300 Mpc/h slab, two
    random sub-catalogues of the mock's size each, 200 x 100 (r, mu) bins,
    the 540-element multipole vector over r = 20 .. 200 Mpc/h, the
    construction at M = 50 and its predicted errors re-binned as in Table 3.
    Every stage is timed with HIP events on the launch stream."""
    import dataclasses

    import mockgen
    from paper_2205_11852_amd.pipeline import Pipeline, block_rebin_map, multipole_map

    wl = dataclasses.replace(mockgen.WORKLOADS["slab"], n_mock=args.slab_mocks)
    t0 = time.perf_counter()
    cats = mockgen.make_catalogues(wl)
    log("[slab] generated %d slabs, %d points in %.1f s" % (wl.n_mock, cats.xyz.shape[1],
                                                            time.perf_counter() - t0))
    pl = Pipeline(cats)
    tuned = None
    if not args.no_autotune:
        tuned = pl.autotune(args.tune_sample)
        log("[slab] autotune: %s" % json.dumps(tuned))
    b = pl.binning
    r_lo = int(round(20.0 / (wl.r_max_mpc / wl.n_r)))
    g540, w540, P540 = multipole_map(b.n_r, b.n_mu, 1, r_lo, b.n_r)
    names = ["cells", "count", "xi", "map", "covariance"]

    def step(ev=None):
        def mark(i):
            if ev:
                ev[i].record(stream)
        mark(0)
        pl.build_cells()
        mark(1)
        pl.count()
        mark(2)
        pl.xi_multipoles()
        mark(3)
        x540 = pl.map_vectors(pl.xi, g540, w540, P540)
        mark(4)
        A, B, C, _ = pl.covariance_general(x540, P540, 0, 1.0, 2.0, 50.0, lc.LC_FP32_MFMA, report=False)
        mark(5)
        return A, B, C

    step()
    torch.cuda.synchronize()
    times = {k: [] for k in names}
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        A, B, C = step(ev)
        torch.cuda.synchronize()
        for i, nm in enumerate(names):
            times[nm].append(ev[i].elapsed_time(ev[i + 1]))
        log("[slab] step %d done" % k)
    wall = (time.perf_counter() - t0) / args.steps
    st = pl.stats_host()
    count_s = float(np.mean(times["count"])) / 1e3
    rep = lc.lc_covariance_general(pl.map_vectors(pl.xi, g540, w540, P540), wl.n_mock, P540, 0, 1.0, 2.0, 50.0,
                                   lc.LC_FP32_MFMA, A, B, C, report=True)
    # Table 3's layout: chi^2_2, cost and iFoM of both estimators for several
    # M and bin widths, from A and B re-binned as matrices (Sect. 5.3)
    table = []
    for dr in (1, 2, 5, 10, 20):
        gb, wb, Pb = block_rebin_map(3, P540 // 3, dr)
        Ab, Bb = pl.map_matrix(A, gb, wb, Pb), pl.map_matrix(B, gb, wb, Pb)
        for M in (10.0, 20.0, 50.0, 100.0):
            r = lc.lc_covcov(Ab, Bb, Pb, 1, M, None, 0, None, None)
            table.append({"M": M, "dr_mpc": dr * wl.r_max_mpc / wl.n_r, "chi2_2_smp": r["chi2_2_smp"],
                          "chi2_2_lc": r["chi2_2_lc"], "ifom_smp": r["ifom_smp"], "ifom_lc": r["ifom_lc"],
                          "gain": r["gain"]})
    achieved = st["binned"] * OPS_PER_BINNED_PAIR / count_s
    return {"workload": "slab: %d mocks x ~%g clustered points in an open 1500x1500x300 Mpc/h slab, two "
                        "random sub-catalogues of the mock's size each, %d r-bins to %g Mpc/h x %d mu-bins, "
                        "z line of sight; 540-element multipole vector (r = 20-200 Mpc/h)"
                        % (wl.n_mock, wl.n_mean, wl.n_r, wl.r_max_mpc, wl.n_mu),
            "mocks_per_hour": wl.n_mock * 3600.0 / wall, "ms_per_step": wall * 1e3,
            "stage_ms": {k: float(np.mean(v)) for k, v in times.items()},
            "pair_tests_per_s": st["candidates"] / count_s, "binned_pairs_per_s": st["binned"] / count_s,
            "binned_pairs_per_step": st["binned"],
            "count_roofline_frac": achieved / PEAK_OPS, "autotuned": tuned,
            "cells": pl.cells.info()["grid"], "check_report": rep, "table3_like": table,
            "note": "A and B from %d synthetic mocks stand in for the paper's 5000 PINOCCHIO slabs; "
                    "chi^2_2 normalised by C = A + B/M" % wl.n_mock}


def covariance_precision(args, torch, lc) -> dict:
    """The covariance-precision workload (c5: 5000 mocks of 5e4 points, the
    40 x 50 (r, mu) vector plus multipoles, P = 2120): counts and data vectors
    on the GPU, then the covariance with float32-MFMA products against the
    float64 path on the same vectors: relative Frobenius error of C^LC, A and
    B, and the error of the extreme eigenvalues of each block of C^LC."""
    import dataclasses

    import mockgen
    from paper_2205_11852_amd.pipeline import Pipeline

    wl = dataclasses.replace(mockgen.WORKLOADS["c5"], n_mock=args.c5_mocks)
    t0 = time.perf_counter()
    cats = mockgen.make_catalogues(wl)
    log("[c5] generated %d mocks, %d points in %.1f s" % (wl.n_mock, cats.xyz.shape[1], time.perf_counter() - t0))
    pl = Pipeline(cats)
    stream = torch.cuda.current_stream()
    pl.build_cells()
    pl.count()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pl.count()
    e1.record(stream)
    pl.xi_multipoles()
    torch.cuda.synchronize()
    count_ms = e0.elapsed_time(e1)
    t = {}
    reps = {}
    for name, prec, checked in (("fp32_mfma", lc.LC_FP32_MFMA, lc.LC_FP32_MFMA_CHECKED),
                                ("fp32_mfma_acc32", lc.LC_FP32_MFMA | lc.LC_ACC32,
                                 lc.LC_FP32_MFMA_CHECKED | lc.LC_ACC32),
                                ("fp64", lc.LC_FP64, lc.LC_FP64)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pl.covariance(prec, report=False)
        b.record(stream)
        torch.cuda.synchronize()
        t[name] = a.elapsed_time(b)
        # the report: the check of C^LC, and for float32 its float64 twin's errors
        reps[name] = pl.covariance(checked, report=True)
    r32, r64 = reps["fp32_mfma"], reps["fp64"]

    def eig_err(r):
        e = []
        for blk in range(2):
            scale = max(abs(r64["min_eig"][blk]), abs(r64["max_eig"][blk]))
            e.append(max(abs(r["min_eig"][blk] - r64["min_eig"][blk]),
                         abs(r["max_eig"][blk] - r64["max_eig"][blk])) / scale)
        return e

    eig = eig_err(r32)
    r32a = reps["fp32_mfma_acc32"]
    eig_a = eig_err(r32a)
    return {"workload": "c5: %d mocks x Poisson(%g), %g Mpc/h periodic box, %d x %d randoms, %d x %d bins, P = %d"
                        % (wl.n_mock, wl.n_mean, wl.box_mpc, wl.n_subsets, wl.subset_size, wl.n_r, wl.n_mu,
                           pl.binning.P),
            "pair_count_ms": count_ms, "mocks_per_hour_pair_count": wl.n_mock * 3600.0 / (count_ms / 1e3),
            "covariance_ms": t, "rel_frob_fp32_vs_fp64": {"C": r32["rel_frob_vs_fp64"][0],
                                                          "A": r32["rel_frob_vs_fp64"][1],
                                                          "B": r32["rel_frob_vs_fp64"][2]},
            "max_eig_error_rel": {"xi_block": eig[0], "multipole_block": eig[1]},
            "fp32_accumulation_over_all_mocks": {
                "note": "float32 MFMA products accumulated in float32 over all %d mocks (LC_ACC32) instead of "
                        "float32 blocks of 256 mocks summed in float64" % wl.n_mock,
                "rel_frob_fp32_vs_fp64": {"C": r32a["rel_frob_vs_fp64"][0], "A": r32a["rel_frob_vs_fp64"][1],
                                          "B": r32a["rel_frob_vs_fp64"][2]},
                "max_eig_error_rel": {"xi_block": eig_a[0], "multipole_block": eig_a[1]},
                "covariance_ms": t["fp32_mfma_acc32"]},
            "report_fp32": r32, "report_fp64": r64}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--mocks", type=int, default=0, help="override the number of mocks")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-mock", action="store_true")
    ap.add_argument("--cell-mpc", type=float, default=0.0)
    ap.add_argument("--sub", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--direct-mocks", type=int, default=8,
                    help="mocks timed for the direct estimate over every random sub-catalogue (0: skip)")
    ap.add_argument("--tune-sample", type=int, default=64, help="tasks timed by the autotuner")
    ap.add_argument("--slab-mocks", type=int, default=100,
                    help="mocks of the paper-shaped slab workload timed after the main line (0: skip)")
    ap.add_argument("--c5-mocks", type=int, default=5000,
                    help="mocks of the covariance-precision workload (c5) reported after the main line (0: skip)")
    ap.add_argument("--slab-only", action="store_true",
                    help="time only the paper-shaped slab workload and print its JSON object (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this path has no multi-GPU mode "
              "(mocks would shard across GPUs with one covariance reduction at the end)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import mockgen
    from paper_2205_11852_amd import lc
    from paper_2205_11852_amd.pipeline import Pipeline

    if args.slab_only:
        print(json.dumps(paper_slab(args, torch, lc, torch.cuda.current_stream())))
        return

    wl = mockgen.WORKLOADS[args.config]
    n_mock = args.mocks or wl.n_mock
    t0 = time.perf_counter()
    log("[bench] generating %s with %d mocks" % (wl.name, n_mock))
    cats = mockgen.make_catalogues(wl, n_mock, progress=log)
    gen_s = time.perf_counter() - t0
    log("[bench] generated %d points in %.1f s" % (cats.xyz.shape[1], gen_s))
    # host -> device copy of the int32 catalogues (outside the timed steps:
    # the path starts from device-resident catalogues)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl = Pipeline(cats)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    cell_units = int(args.cell_mpc * mockgen.UNITS_PER_MPC)
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_autotune and cell_units == 0 and args.sub == 0:
        # mesh and launch shape chosen by timing a sample of the tasks (once,
        # outside the timed region; the library caches the choice)
        t0 = time.perf_counter()
        tuned = pl.autotune(args.tune_sample)
        log("[bench] autotune: %s (%.1f s)" % (json.dumps(tuned), time.perf_counter() - t0))

    def step(events=None):
        # events: step start, mesh built, counted, xi, covariance and check
        if events:
            events[0].record(stream)
        pl.build_cells(cell_units, args.sub)
        if events:
            events[1].record(stream)
        pl.count()
        if events:
            events[2].record(stream)
        pl.xi_multipoles()
        if events:
            events[3].record(stream)
        rep = pl.covariance(lc.LC_FP32_MFMA, report=True)
        if events:
            events[4].record(stream)
        return rep

    for w in range(args.warmup):
        log("[bench] warmup step %d" % w)
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = None
    for k in range(args.steps):
        rep = step(evs[k])
        log("[bench] step %d done" % k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    count_ms = [e[1].elapsed_time(e[2]) for e in evs]
    stage_ms = {name: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs]))
                for i, name in enumerate(("cells", "count", "xi", "covariance_and_check"))}
    st = pl.stats_host()
    binned = st["binned"]
    cand = st["candidates"]
    kern_s = float(np.mean(count_ms)) / 1e3
    ms_per_step = wall / args.steps * 1e3
    mocks_per_hour = n_mock * 3600.0 / (wall / args.steps)
    achieved = binned * OPS_PER_BINNED_PAIR / kern_s

    out = {
        "metric": METRIC,
        "value": mocks_per_hour,
        "unit": "mocks/hour",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64/f64 (pair counts exact; covariance f32-MFMA products, f64 combination)",
        "data": "synthetic (seeded Neyman-Scott mocks and uniform randoms)",
        "config": {"workload": workload_text(wl, n_mock),
                   "n_tasks": int(len(pl.tasks)), "cells": pl.cells.info()["grid"],
                   "sub_cells": pl.cells.info()["sub"], "autotuned": tuned},
        "pair_tests_per_s": cand / kern_s,
        "binned_pairs_per_s": binned / kern_s,
        "pair_count_ms": float(np.mean(count_ms)),
        "stage_ms": stage_ms,
        "inputs": {"generation_s": gen_s, "h2d_s": h2d_s, "h2d_bytes": int(cats.xyz.nbytes),
                   "note": "synthetic catalogues drawn on the host and copied once; not part of a step"},
        "candidates_per_step": cand,
        "binned_pairs_per_step": binned,
        "exact_fallback_fraction": st["exact_fallback"] / max(binned, 1),
        "check_report": rep,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / PEAK_OPS,
                     "traffic": measured_traffic(args.config, n_mock, wl.n_mock)},
    }

    if not args.no_per_mock:
        # Batched (one persistent launch), the same launch replayed from a
        # captured hipGraph, and the per-mock baseline (one launch per task,
        # mock after mock, a synchronisation after each mock), each run once
        # untimed and then timed as the median of a few wall-clock runs.
        def wall(fn, reps):
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return float(np.median(ts)), ts

        def compare(p, reps):
            p.count()
            torch.cuda.synchronize()
            ref = p.counts.clone()
            p.count_per_mock()
            p.count(lc.LC_GRAPH)
            torch.cuda.synchronize()
            tb, tbs = wall(p.count, reps)
            tg, tgs = wall(lambda: p.count(lc.LC_GRAPH), reps)
            same = bool(torch.equal(ref, p.counts))
            tp, tps = wall(p.count_per_mock, reps)
            same = same and bool(torch.equal(ref, p.counts))
            return {"batched_s": tb, "graph_replay_s": tg, "per_mock_s": tp, "speedup": tp / tb,
                    "speedup_graph": tp / tg, "runs": reps, "batched_runs_s": tbs, "graph_runs_s": tgs,
                    "per_mock_runs_s": tps, "counts_identical": same}

        log("[bench] batched vs per-mock (%s)" % wl.name)
        out["batched_vs_per_mock"] = dict(workload=wl.name, **compare(pl, 3))
        if args.config != "c1":
            # the small workload, where launch overhead dominates
            c1 = mockgen.make_catalogues(mockgen.WORKLOADS["c1"])
            p1 = Pipeline(c1)
            p1.build_cells()
            log("[bench] batched vs per-mock (c1)")
            out["batched_vs_per_mock_c1"] = dict(workload="c1", **compare(p1, 5))
            del p1

    # predicted error of the covariance estimates at M = 50 (Sect. 3, 5.3)
    out["covcov_M50"] = pl.covcov(50.0)

    if args.direct_mocks > 0 and not cats.wl.per_mock_randoms:
        # The cost the linear construction avoids (Sect. 2.3, Table 3): the
        # direct split estimate over all M random sub-catalogues needs DD and M
        # DR per mock (plus each RR once), against DD, DR1, DR2 for LC.
        from paper_2205_11852_amd.pipeline import plan_direct_tasks
        subsets = cats.random_catalogue_ids()
        M = len(subsets)
        nd = min(args.direct_mocks, n_mock)
        log("[bench] direct estimate: %d mocks x M = %d" % (nd, M))
        tasks_d, _ = plan_direct_tasks(range(nd), subsets)
        parts = {"rr": tasks_d[:M], "dd_dr": tasks_d[M:]}
        t_ms = {}
        for key, tk in parts.items():
            cd = torch.zeros((len(tk), pl.binning.n_r, pl.binning.n_mu), dtype=torch.int64, device="cuda")
            tune = pl.tuned["tune"] if pl.tuned else None
            lc.lc_pair_count_batch(pl.cells, tk, pl.binning, cd, lc.LC_PERSISTENT, tune, None)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lc.lc_pair_count_batch(pl.cells, tk, pl.binning, cd, lc.LC_PERSISTENT, tune, None)
            e1.record(stream)
            torch.cuda.synchronize()
            t_ms[key] = e0.elapsed_time(e1)
            del cd
        direct = t_ms["dd_dr"] / 1e3 / nd + t_ms["rr"] / 1e3 / n_mock
        lc_mock = kern_s / n_mock
        nbar = float(np.mean(pl.sizes[:n_mock]))
        ns = float(wl.subset_size)
        model = (0.5 * nbar * nbar + M * nbar * ns) / (0.5 * nbar * nbar + 2 * nbar * ns)
        out["direct_vs_lc"] = {"M": M, "mocks_timed": nd, "direct_pair_count_s_per_mock": direct,
                               "lc_pair_count_s_per_mock": lc_mock, "ratio": direct / lc_mock,
                               "pair_ratio_model": model,
                               "note": "RR of the shared sub-catalogues amortised over all mocks in both"}

    if args.c5_mocks > 1:
        log("[bench] covariance precision (c5)")
        out["covariance_precision_c5"] = covariance_precision(args, torch, lc)

    if args.slab_mocks > 0:
        log("[bench] paper-shaped slab workload")
        out["paper_slab"] = paper_slab(args, torch, lc, stream)

    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        log("[bench] cpu baseline (oracle) on mock 0")
        e = pl.est[0]
        D, R1, R2 = pl.tasks[e[0]][0], pl.tasks[e[1]][1], pl.tasks[e[2]][1]
        n_d = int(pl.sizes[D])
        full = n_d * (n_d - 1) / 2 + n_d * float(pl.sizes[R1] + pl.sizes[R2])
        # RR per mock: a shared sub-catalogue's RR is counted once for the
        # whole batch, per-mock sub-catalogues once per mock
        rr_tests = sum(float(pl.sizes[pl.tasks[t][0]]) * (pl.sizes[pl.tasks[t][0]] - 1) / 2
                       for t in set(pl.est[:, 3:].ravel().tolist())) / n_mock
        t0 = time.perf_counter()
        if full <= CPU_SAMPLE_TESTS:
            for a, b in ((D, None), (D, R1), (D, R2)):
                oracle.count_pairs(cats.cat(a), None if b is None else cats.cat(b), wl.r_edges_units, wl.n_mu,
                                   wl.box_units, wl.los)
            tests = full
            what = "brute-force DD, DR1, DR2 of mock 0"
        else:
            # a bounded sample: the first n_s points of mock 0 against all of
            # mock 0, R1 and R2 (every test costs the same in the oracle)
            n_s = max(1, int(CPU_SAMPLE_TESTS / (n_d + float(pl.sizes[R1] + pl.sizes[R2]))))
            head = cats.cat(D)[:, :n_s]
            for b in (D, R1, R2):
                oracle.count_pairs(head, cats.cat(b), wl.r_edges_units, wl.n_mu, wl.box_units, wl.los)
            tests = n_s * (n_d + float(pl.sizes[R1] + pl.sizes[R2]))
            what = ("brute-force cross counts of %d points of mock 0 against mock 0, R1 and R2, "
                    "scaled to the %.2e tests of its DD, DR1, DR2" % (n_s, full))
        t_cpu = time.perf_counter() - t0
        rate = tests / t_cpu
        t_mock = (full + rr_tests) / rate
        out["cpu_baseline"] = {"value": 3600.0 / t_mock, "unit": "mocks/hour",
                               "cores": oracle.threads_used(), "kind": "oracle",
                               "sample": "%s (%.2e pair tests, %.1f s) plus its share of the RR counts; "
                                         "LS/covariance excluded" % (what, tests, t_cpu),
                               "pair_tests_per_s": rate}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
