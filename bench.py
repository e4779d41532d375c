#!/usr/bin/env python
"""Throughput of the CONCORD proximal-gradient iteration on one MI355X.

Workload: the Obs form (Y = Omega X^T, gradient from Y X / n) at p = 20,000
variables, n = 5,000 observations; true Omega0 random with 10 off-diagonal
nonzeros per row, values +-U[0.1, 0.3], diagonal = row abs-sum + 0.1; rows of
X ~ N(0, Omega0^{-1}), columns standardised; lambda1 = 0.4, lambda2 = 0.05.

A step is one outer iteration of the method: the dense gradient contraction
(MFMA), the candidate set, the batched step-size trials with the
sufficient-decrease test, CSR emission of the accepted iterate and the
product refresh Y = Omega X^T with the objective sums.  Inputs are resident in
HBM before the timed region.  Both precision forms are timed (BF16 hi/lo split
and plain FP32); ``value`` is the BF16-split form.

Prints one JSON line.  --gpus N with N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "prox-grad iters/sec + HBM/MFMA roofline fraction at p=20k; BF16-split vs FP32"
PEAK_TFLOPS = {"bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def stream_copy_gbps(torch, mib=2048, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of torch's copy kernel
    on two buffers of `mib` MiB: the achievable HBM rate that HBM-bound kernels are
    also compared with (alongside the 8 TB/s peak)."""
    src = torch.empty(mib * 262144, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * mib * 1048576 / (ms * 1e-3) / 1e9


def environment(torch, seed):
    """What the run was measured on: software versions, the device and the workload's seed
    (the clocks under this load are in the headline profile's power section)."""
    from paper_1710_10769_amd._lib import concord_version
    prop = torch.cuda.get_device_properties(0)
    return {"library": concord_version(), "torch": torch.__version__, "hip": torch.version.hip,
            "device": getattr(prop, "gcnArchName", prop.name),
            "compute_units": prop.multi_processor_count, "seed": seed}


def run_form(torch, X32, p, n, lam1, lam2, form, steps, warmup):
    from paper_1710_10769_amd import Solver
    s = Solver(p, n, variant="obs", precision=form)
    s.set_data(X32)
    log(f"{form}: warmup {warmup} steps")
    for _ in range(warmup):
        s.step(lam1, lam2)
    s.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [s.step(lam1, lam2) for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile()
    s.set_profiling(False)
    log(f"{form}: {steps} steps in {t1 - t0:.3f} s")
    variant = s.contraction_variant()[1]
    om = s.get_omega_scipy()
    s.close()
    sec = t1 - t0
    dense_ms, dense_n = prof["dense"]
    gemm_ms = dense_ms / max(dense_n, 1)
    flops = 2.0 * n * p * p   # algorithmic flops of Y X / n per iteration
    achieved = flops / (gemm_ms * 1e-3) / 1e12
    res = {
        "value": steps / sec,
        "ms_per_step": sec / steps * 1e3,
        "kernel_ms_per_step": {k: v[0] / steps for k, v in prof.items()},
        "dense_kernel_avg_ms": gemm_ms,
        "contraction_variant": variant,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[form],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[form],
                     "traffic": stored_traffic(form, variant),
                     # the BF16 split runs three BF16 products (hi*hi, hi*lo, lo*hi) per
                     # useful flop: the rate the matrix cores actually execute
                     "executed_per_useful_flop": 3 if form == "bf16x3" else 1,
                     "frac_executed": achieved * (3 if form == "bf16x3" else 1) / PEAK_TFLOPS[form]},
        "trials_per_step": sum(i.n_trials for i in infos) / steps,
        "final_F": infos[-1].F,
        "final_nnz": infos[-1].nnz,
    }
    return res, om


def run_cov_context(torch, X32, p, n, lam1, lam2, steps, warmup):
    """The Cov form on the same data: S = X^T X / n formed once (timed apart), then
    the same outer iterations from Omega = I.  Context for the choice between the two
    forms (Lemma 3.1); not the headline."""
    from paper_1710_10769_amd import Solver
    s = Solver(p, n, variant="cov", precision="bf16x3")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_data(X32)
    torch.cuda.synchronize()
    form_s = time.perf_counter() - t0
    for _ in range(warmup):
        s.step(lam1, lam2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [s.step(lam1, lam2) for _ in range(steps)]
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    om = s.get_omega_scipy()
    # the phase breakdown from the same steps replayed with the per-phase HIP events on
    # (untimed: the events cost a few microseconds each, a large part of a 0.2 ms step)
    s.reset()
    for _ in range(warmup):
        s.step(lam1, lam2)
    s.set_profiling(True)
    for _ in range(steps):
        s.step(lam1, lam2)
    prof = s.profile()
    s.close()
    log(f"cov context: {steps} steps in {sec:.3f} s, S formed in {form_s * 1e3:.1f} ms")
    return {"variant": "cov", "precision": "bf16x3", "value": steps / sec, "unit": "iters/s",
            "ms_per_step": sec / steps * 1e3, "s_formation_ms": form_s * 1e3,
            "kernel_ms_per_step": {k: v[0] / steps for k, v in prof.items()},
            "final_F": infos[-1].F, "final_nnz": infos[-1].nnz}, om


def stored_traffic(form, variant, record="traffic_gemm_sym_obs_p20000_n5000.json",
                   want_form="bf16x3"):
    """HBM bytes per launch of a kernel from a committed counter record under profiles/, or
    None when the record is for another form or tile variant, or the kernel's source
    changed since the counters were taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", record)
    if form != want_form or not os.path.exists(rec_path):
        return None
    rec = json.load(open(rec_path))
    if rec.get("variant", variant) != variant:
        return None
    src = os.path.join(ROOT, rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes"]


def cpu_baseline(X64, lam1, lam2):
    """The FP64 oracle, untuned, on one full-size outer iteration of the workload."""
    import numpy as np  # noqa: F401
    import threadpoolctl
    from oracle import concord as oc
    t0 = time.perf_counter()
    oc.solve(lam1, lam2, "obs", X=X64, fixed_iters=1, check_literal=False)
    sec = time.perf_counter() - t0
    threads = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)
    return {"value": 1.0 / sec, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": "1 outer iteration at the full workload size (p=20000, n=5000), FP64 "
                      "NumPy/SciPy; dense BLAS multithreaded, sparse products single-threaded",
            "seconds": sec}


def bench_c1(args, torch, np, datagen):
    """Small Cov FP64 solve (p = 200, n = 100, chain graph; lambda1 0.3, lambda2 0.1,
    tol 1e-5 / 200 iterations): launch-latency bound, so it is reported with and
    without graph replay and on the device-resident loop.  A step is one whole solve;
    value = iterations/s of the handle's default (direct launches)."""
    from paper_1710_10769_amd import Solver
    w = datagen.make_workload("c1_cov_fp64_p200")
    X = torch.from_numpy(w.X).cuda()
    out = {}
    for g in (False, True):
        s = Solver(w.p, w.n, variant="cov", precision="fp64", use_graph=g)
        s.set_data(X)
        times, iters = [], 0
        for rep in range(args.warmup + args.steps):
            s.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            si = s.solve(w.lam1, w.lam2, w.tol, w.max_iter)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append(time.perf_counter() - t0)
                iters = si.iters
        s.close()
        out[g] = (iters, float(np.median(times)))
        log(f"graph={g}: {iters} iterations in {out[g][1] * 1e3:.3f} ms")
    # the same solve on the device-resident batched path (a batch of one): the iteration
    # control stays on the device, the host reads two counters per replay of K iterations
    from paper_1710_10769_amd import Batch
    dev = {}
    for K in (4, 8):
        b = Batch([X], [w.lam1], precision="fp64", iters_per_launch=K)
        times = []
        for rep in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iters_b, _, _ = b.solve(w.lam2, w.tol, w.max_iter)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append(time.perf_counter() - t0)
        st = b.stats()
        b.close()
        dev[K] = {"iters_per_s": iters_b[0] / float(np.median(times)),
                  "ms_per_solve": float(np.median(times)) * 1e3, "iterations": iters_b[0],
                  "replays": st["launches"], "host_syncs": st["host_syncs"]}
        log(f"device loop K={K}: {dev[K]}")
    it, sec = out[False]
    line = {
        "metric": "prox-grad iters/sec, Cov FP64 p=200 (launch-latency bound)",
        "value": it / sec, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cov_chain_p200_n100", "p": w.p, "n": w.n, "lam1": w.lam1,
                   "lam2": w.lam2, "iterations": it},
        "with_graph": {"value": out[True][0] / out[True][1], "ms_per_solve": out[True][1] * 1e3},
        "device_loop": {f"iters_per_launch_{k}": v for k, v in dev.items()},
    }
    print(json.dumps(line), flush=True)


def timed_solve(torch, s, lam1, lam2, tol, max_iter):
    """A solve from Omega = I timed without profiling (the per-phase HIP events cost a few
    microseconds each, a third of an iteration at p = 16,384), after an untimed one that
    takes the handle's first-use allocations."""
    s.solve(lam1, lam2, tol, max_iter)
    s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    si = s.solve(lam1, lam2, tol, max_iter)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, si


def profiled_solve(s, lam1, lam2, tol, max_iter):
    """The same solve once more with the per-phase HIP events on: the phase breakdown."""
    s.reset()
    s.set_profiling(True)
    s.solve(lam1, lam2, tol, max_iter)
    prof = s.profile()
    s.set_profiling(False)
    return prof


def bench_c3(args, torch, np, datagen):
    """Cov precision forms at p = 16,384, n = 4,096 (random degree 8; lambda1 0.3,
    lambda2 0.1, tol 1e-5 / 200): S formed once on MFMA, then the solve.  Each
    form is timed; its final Omega is compared with the FP64 form's."""
    from paper_1710_10769_amd import Solver
    log("generating c3 workload")
    w = datagen.make_workload("c3_cov_p16384", backend="torch", device="cuda")
    X32 = torch.from_numpy(w.X.astype(np.float32)).cuda()
    X64 = X32.double()
    res, oms = {}, {}
    for form in ("fp64", "fp32", "bf16x3"):
        s = Solver(w.p, w.n, variant="cov", precision=form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_data(X64 if form == "fp64" else X32)
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        t_solve, si = timed_solve(torch, s, w.lam1, w.lam2, w.tol, w.max_iter)
        prof = profiled_solve(s, w.lam1, w.lam2, w.tol, w.max_iter)
        oms[form] = s.get_omega_scipy()
        # untimed replay of the same iterates counting, for every refresh of the solve (one
        # at Omega = I, one per accepted step), the tile pairs that passed the screening
        s.reset()
        act_total, nref, npairs = 0, 0, 0
        for k in range(si.iters + 1):
            npairs, act = s.refresh_screen_stats(w.lam1)
            act_total += act
            nref += 1
            if k < si.iters:
                s.step(w.lam1, w.lam2)
        s.close()
        ref_ms = prof["refresh"][0] / max(prof["refresh"][1], 1)
        eb = 8 if form == "fp64" else 4
        # the refresh kernel forms M = (Omega S + S Omega) / 2 for the tile pairs kept by
        # the screening and writes their candidate threshold words (the screening zeroes
        # the rest).  Algorithmic bytes per launch: the S tiles of the kept pairs (two
        # 64 x 64 tiles per off-diagonal pair, one per diagonal pair) plus their words
        # (64 rows x 8 bytes per tile); S rows re-read per nonzero of Omega come from
        # L2/MALL.  Timed alone (class "refresh").
        T = (w.p + 63) // 64
        tiles = (2 * (act_total - nref * T) + nref * T) / nref
        s_bytes = tiles * 64 * 64 * eb
        words_b = tiles * 64 * 8.0
        gbs = (s_bytes + words_b) / (ref_ms * 1e-3) / 1e9
        res[form] = {"iters": si.iters, "iters_per_s": si.iters / t_solve, "solve_s": t_solve,
                     "s_formation_s": t_s, "nnz": si.nnz, "F": si.F,
                     "refresh_ms": ref_ms, "refresh_GBps": gbs,
                     "refresh_pairs_loading_S_frac": act_total / (nref * npairs),
                     "refresh_algorithmic_MB": (s_bytes + words_b) / 1e6,
                     "kernel_ms_per_iter": {k: v[0] / max(si.iters, 1) for k, v in prof.items()}}
        log(f"{form}: {si.iters} iterations, {t_solve:.3f} s, S in {t_s:.3f} s")
    # the BF16x3 form once more with the screening off: the refresh then forms every tile
    # pair (the plain product of Algorithm 2), reading all of S each iteration
    s = Solver(w.p, w.n, variant="cov", precision="bf16x3", screen=False)
    s.set_data(X32)
    t_solve, si = timed_solve(torch, s, w.lam1, w.lam2, w.tol, w.max_iter)
    prof = profiled_solve(s, w.lam1, w.lam2, w.tol, w.max_iter)
    same = bool((s.get_omega_scipy() != oms["bf16x3"]).nnz == 0)
    s.close()
    ref_ms = prof["refresh"][0] / max(prof["refresh"][1], 1)
    unscreened = {"iters": si.iters, "iters_per_s": si.iters / t_solve, "F": si.F,
                  "same_omega_as_screened": same, "refresh_ms": ref_ms,
                  # every pair: S read once (p^2 entries, 4 bytes) + p^2 / 8 bytes of words
                  "refresh_GBps": (w.p * w.p * 4.0 + w.p * w.p / 8.0) / (ref_ms * 1e-3) / 1e9,
                  "kernel_ms_per_iter": {k: v[0] / max(si.iters, 1) for k, v in prof.items()}}
    log(f"bf16x3 unscreened: {si.iters} iterations, {t_solve:.3f} s")
    ref = oms["fp64"]
    scale = float(np.abs(ref.data).max())
    for form in ("fp32", "bf16x3"):
        d = oms[form] - ref
        res[form]["max_abs_diff_vs_fp64_rel"] = (float(np.abs(d.data).max()) if d.nnz else 0.0) / scale
        g, r = oms[form].copy(), ref.copy()
        g.data[:] = 1; r.data[:] = 1
        res[form]["support_mismatches_vs_fp64"] = int((abs(g - r)).nnz)
    copy_gbps = stream_copy_gbps(torch)
    ref_gbps = res["bf16x3"]["refresh_GBps"]
    line = {
        "metric": "Cov prox-grad iters/sec at p=16,384 per precision form",
        "value": res["bf16x3"]["iters_per_s"], "unit": "iters/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": 1e3 / res["bf16x3"]["iters_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": "cov_random_deg8_p16384_n4096", "p": w.p, "n": w.n,
                   "lam1": w.lam1, "lam2": w.lam2, "tol": w.tol},
        "forms": res,
        "bf16x3_unscreened": unscreened,
        # the unscreened refresh is a plain streaming pass over S: its rate against the peak
        "roofline_unscreened": {"bound": "hbm", "kernel": "cov_refresh_kernel",
                                "achieved": unscreened["refresh_GBps"], "peak": 8000.0,
                                "unit": "GB/s", "frac": unscreened["refresh_GBps"] / 8000.0},
        # the Cov refresh kernel of the BF16x3 form: the S tiles (packed hi|lo, 4 bytes an
        # entry) of the pairs kept by the screening, read once, and their threshold words
        "roofline": {"bound": "hbm", "kernel": "cov_refresh_kernel", "achieved": ref_gbps,
                     "peak": 8000.0, "unit": "GB/s", "frac": ref_gbps / 8000.0,
                     "traffic": stored_traffic("bf16x3", None,
                                               record="traffic_cov_refresh_c3_p16384.json"),
                     "stream_copy_GBps": copy_gbps,
                     "frac_of_stream_copy": ref_gbps / copy_gbps},
    }
    print(json.dumps(line), flush=True)


def bench_c6(args, torch, np, datagen):
    """fMRI-shaped Cov stand-in (Section 5): p = 91,282 in three spatial kNN blocks,
    n = 5,142, FP32.  S = X^T X / n (33 GB) is formed once on MFMA, then the lambda1
    column of the paper's grid at lambda2 = 0.10 is solved from Omega = I per point
    (tol 1e-5, 200 iterations at most).  The standardised X is scaled by c so that
    the estimate turns diagonal only above lambda1 = 0.80 at lambda2 = 0.10: the
    covariance's own scale is not given, and by the scaling identity c only selects
    which part of the lambda path the paper's grid samples."""
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.path import average_degree, scale_for_lambda_grid, support_recovery
    torch.backends.cuda.matmul.allow_tf32 = False
    log("generating c6 workload (spatial kNN blocks, B B^T + CG sampler)")
    t0 = time.perf_counter()
    kw = {}
    if args.scale != 1.0:
        kw = dict(p=int(91282 * args.scale), n=max(64, int(5142 * args.scale)))
    w = datagen.make_workload("c6_fmri_cov_p91282", backend="torch", device="cuda", **kw)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    p, n = w.p, w.n
    X = torch.from_numpy(w.X.astype(np.float32)).cuda()
    om0 = w.omega0
    del w
    # largest off-diagonal |s_ij| of the standardised data, in row blocks
    m = 0.0
    for r0 in range(0, p, 8192):
        r1 = min(p, r0 + 8192)
        blk = (X[:, r0:r1].T @ X) / n
        idx = torch.arange(r1 - r0, device=X.device)
        blk[idx, idx + r0] = 0.0
        m = max(m, float(blk.abs().max()))
        del blk
    b = min(datagen.FMRI_LAMBDA2)
    c = scale_for_lambda_grid(m, 0.80, b)
    X *= c
    log(f"max off-diagonal |s_ij| {m:.4f}; scale c = {c:.4f}")
    s = Solver(p, n, variant="cov", precision="fp32")
    s.set_data(X)                  # tunes the S contraction for this shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_data(X)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    lam2 = b
    points = []
    t_all = 0.0
    est_first = None
    for lam1 in datagen.FMRI_LAMBDA1:
        s.reset()
        dt, si = timed_solve(torch, s, lam1, lam2, 1e-5, 200)
        t_all += dt
        est = s.get_omega_scipy()
        prof = profiled_solve(s, lam1, lam2, 1e-5, 200)
        deg = average_degree(est)
        points.append({"lam1": lam1, "iters": si.iters, "seconds": dt, "nnz": si.nnz, "F": si.F,
                       "avg_degree": deg,
                       "ms_per_iter": {k: v[0] / max(si.iters, 1) for k, v in prof.items()}})
        log(f"lambda1 {lam1}: {si.iters} iterations, {dt:.2f} s, degree {deg:.2f}")
        if lam1 == min(datagen.FMRI_LAMBDA1):
            est_first = est
    # untimed replay of the densest point: tile pairs kept by the screening and the nonzeros
    # of each iterate the refresh runs at
    lam_first = min(datagen.FMRI_LAMBDA1)
    s.reset()
    replay = []
    it_first = [q["iters"] for q in points if q["lam1"] == lam_first][0]
    for k in range(it_first + 1):
        npairs, act = s.refresh_screen_stats(lam_first)
        replay.append({"iterate": k, "nnz": s.nnz(), "pairs_loading_S": act,
                       "frac": act / npairs})
        if k < it_first:
            s.step(lam_first, lam2)
    # support recovery at the densest point of the column (smallest lambda1), and edges
    # between blocks there
    rec = support_recovery(est_first, om0)
    blocks = datagen.fmri_blocks(args.scale)
    bounds = np.cumsum([0] + [mm for _, mm in blocks])
    e = sp_triu_coo(est_first)
    blk_r = np.searchsorted(bounds, e[0], side="right")
    blk_c = np.searchsorted(bounds, e[1], side="right")
    s.close()
    iters = sum(q["iters"] for q in points)
    line = {
        "metric": "fMRI-shaped Cov solves/sec at p=91,282 (lambda1 column of the paper's grid)",
        "value": len(points) / t_all, "unit": "solves/s", "n_gpus": 1, "steps": len(points),
        "warmup": 0, "ms_per_step": t_all / len(points) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "cov_spatial_knn6_blocks_p91282_n5142", "p": p, "n": n,
                   "blocks": [mm for _, mm in blocks], "lam1": list(datagen.FMRI_LAMBDA1),
                   "lam2": lam2, "tol": 1e-5, "data_scale": c,
                   "max_offdiag_abs_s_standardised": m},
        "s_formation_s": t_s,
        "iterations_total": iters,
        "ms_per_iteration": t_all / max(iters, 1) * 1e3,
        "full_grid_extrapolated_s": t_all / len(points) * len(datagen.FMRI_LAMBDA1) * len(datagen.FMRI_LAMBDA2),
        "points": points,
        "support_vs_omega0_at_lam1_min": rec,
        "screening_at_lam1_min": replay,
        "cross_block_edges_at_lam1_min": int((blk_r != blk_c).sum()),
        "paper_context": "about 37 minutes per (lambda1, lambda2) pair on a CPU cluster (Section 5)",
    }
    print(json.dumps(line), flush=True)


def sp_triu_coo(m):
    import scipy.sparse as sp
    u = sp.triu(sp.csr_matrix(m), k=1).tocoo()
    keep = u.data != 0
    return u.row[keep], u.col[keep]


def bench_c5(args, torch, np, datagen):
    """Differentiation form at p = 200,000, n = 1,000 (random degree 20), FP32:
    forward f(Omega; X) and backward (d f / d Omega on the stored entries, d f / d X)."""
    import scipy.sparse as sp
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    log("generating c5 workload (B B^T + CG)")
    w = datagen.make_workload("c5_grad_p200000", backend="torch", device="cuda")
    rng = np.random.Generator(np.random.PCG64(505))
    om = sp.csr_matrix(datagen.perturb_symmetric(w.omega0, rng, 0.1))
    rp = torch.from_numpy(om.indptr.astype(np.int64)).cuda()
    cl = torch.from_numpy(om.indices.astype(np.int32)).cuda()
    vals = torch.from_numpy(om.data.astype(np.float32)).cuda()
    X = torch.from_numpy(w.X.astype(np.float32)).cuda()
    s = Solver(w.p, w.n, variant="obs", precision="fp32")
    fw, bw = [], []
    for rep in range(args.warmup + args.steps):
        v = vals.clone().requires_grad_(True)
        x = X.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = concord_smooth(v, x, rp, cl, w.lam2, s)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep >= args.warmup:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    s.close()
    tf, tb = float(np.median(fw)), float(np.median(bw))
    line = {
        "metric": "differentiation form forward+backward per second at p=200,000",
        "value": 1.0 / (tf + tb), "unit": "fwd+bwd/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": (tf + tb) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "obs_grad_random_deg20_p200000_n1000", "p": w.p, "n": w.n,
                   "nnz": int(om.nnz), "lam2": w.lam2},
        "forward_ms": tf * 1e3, "backward_ms": tb * 1e3,
        "note": "forward includes X ingest (transpose to variable-major) and the CSR copy-in",
    }
    print(json.dumps(line), flush=True)


def bench_c4(args, torch, np, datagen):
    """Batched lambda path: 48 Cov instances (p in {1k, 2k, 4k, 8k}, n = p/2), each
    solved at lambda1 in {0.2, 0.3, 0.5} from Omega = I (FP64 reductions, stop at
    relative F change < 1e-5 or 200 iterations), all 144 solves on the device at once
    (graph replays of 4 iterations, device-side control).  A step is one whole path from
    the data (S formation included); value = solves per second with FP32 products, the
    workload's precision (the BF16 split form beside it)."""
    from paper_1710_10769_amd import Batch
    l1s, lam2 = datagen.lambda_path_c4()
    log("generating 48 instances")
    inst = datagen.c4_instances(backend="torch", device="cuda")
    Xs = [torch.from_numpy(X.astype(np.float32)).cuda() for _, X, _ in inst]
    torch.cuda.synchronize()
    nsolve = len(inst) * len(l1s)
    res = {}
    for form in args.c4_forms.split(","):
        times = []
        iters = None
        stats = None
        for rep in range(args.warmup + args.steps):
            b = Batch(Xs, l1s, precision=form, iters_per_launch=args.iters_per_launch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iters, Fs, rc = b.solve(lam2, 1e-5, 200)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            stats = b.stats()
            b.close()
            if rep >= args.warmup:
                times.append(t1 - t0)
            log(f"{form} path {rep}: {t1 - t0:.4f} s (S {stats['s_ms']:.1f} ms, iterations "
                f"{stats['iterate_ms']:.1f} ms, {stats['launches']} replays), max iterations {max(iters)}")
        sec = float(np.mean(times))
        res[form] = {"value": nsolve / sec, "ms_per_step": sec * 1e3,
                     "mean_iterations": float(np.mean(iters)), "max_iterations": int(max(iters)),
                     "total_iterations": int(np.sum(iters)), "last_path": stats}
    head = list(res)[0]
    # autotuned against fixed contraction tiles: one path with one variant forced for every
    # instance shape (the tuner picks per shape key: form, p rounded to 256, K)
    fixed = {}
    if not args.no_fixed_tiles:
        # variants 0 and 1 of the FP32 and BF16-split tables: the 256 x 256 tile on 8 waves
        # and the 128 x 128 tile on 4 waves (the FP64 table has one variant)
        for v in ((0,) if head == "fp64" else (0, 1)):
            os.environ["CONCORD_GEMM_VARIANT"] = str(v)
            try:
                b = Batch(Xs, l1s, precision=head, iters_per_launch=args.iters_per_launch)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.solve(lam2, 1e-5, 200)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = b.stats()
                b.close()
            finally:
                del os.environ["CONCORD_GEMM_VARIANT"]
            name = f"variant_{v}"
            fixed[name] = {"solves_per_s": nsolve / (t1 - t0), "s_ms": st["s_ms"],
                           "iterate_ms": st["iterate_ms"]}
            log(f"{head} fixed contraction {name}: {t1 - t0:.4f} s (S {st['s_ms']:.1f} ms)")
    line = {
        "metric": "batched lambda-path solves/sec (48 Cov instances x 3 lambda1)",
        "value": res[head]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res[head]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
        "config": {"workload": "cov_batched_lambda_path_48x3", "instances": len(inst),
                   "p": [p for p, _, _ in inst], "lambda1": list(l1s), "lam2": lam2},
        **{k: v for k, v in res[head].items() if k not in ("value", "ms_per_step")},
        "other_forms": {k: v for k, v in res.items() if k != head},
        "fixed_contraction_tiles": fixed,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="bf16x3,fp32")
    ap.add_argument("--c4-forms", default="fp32,bf16x3",
                    help="c4: precision forms, the first one is the line's value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cov-context", action="store_true",
                    help="skip timing the Cov form on the same problem")
    ap.add_argument("--no-fixed-tiles", action="store_true",
                    help="c4 only: skip the paths with one contraction variant forced")
    ap.add_argument("--iters-per-launch", type=int, default=4,
                    help="c4 only: iterations captured per graph replay")
    ap.add_argument("--p", type=int, default=20000)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "c6"],
                    help="c2: the Obs p=20k headline; c1: the small Cov FP64 solve; "
                         "c4: the batched lambda path; c3: Cov precision forms; "
                         "c5: differentiation form; c6: fMRI-shaped Cov workload")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="c6 only: shrink the fMRI-shaped workload (blocks and n) by this factor")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import datagen

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib * 262144, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    if args.workload == "c4":
        return bench_c4(args, torch, np, datagen)
    if args.workload == "c1":
        return bench_c1(args, torch, np, datagen)
    if args.workload == "c3":
        return bench_c3(args, torch, np, datagen)
    if args.workload == "c5":
        return bench_c5(args, torch, np, datagen)
    if args.workload == "c6":
        return bench_c6(args, torch, np, datagen)
    p, n = args.p, args.n
    log(f"generating workload p={p} n={n}")
    t0 = time.perf_counter()
    w = datagen.make_workload("c2_obs_p20000", p=p, n=n, backend="torch", device="cuda")
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    X32 = torch.from_numpy(w.X.astype(np.float32)).to("cuda")
    forms = [f for f in args.forms.split(",") if f]
    out = {}
    oms = {}
    for form in forms:
        out[form], oms[form] = run_form(torch, X32, p, n, w.lam1, w.lam2, form, args.steps,
                                        args.warmup)
    head = forms[0]
    line = {
        "metric": METRIC,
        "value": out[head]["value"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"obs_random_deg10_standardized_p{p}_n{n}", "p": p, "n": n,
                   "lam1": w.lam1, "lam2": w.lam2, "variant": "obs", "precision": head,
                   "trial_batch": 8},
        "roofline": out[head]["roofline"],
    }
    for f in forms[1:]:
        line[f] = {k: out[f][k] for k in ("value", "ms_per_step", "roofline", "dense_kernel_avg_ms",
                                           "contraction_variant")}
        line[f"{head}_over_{f}"] = out[head]["value"] / out[f]["value"]
        a, b = oms[head], oms[f]
        d = a - b
        scale = float(np.abs(b.data).max())
        line[f"final_omega_maxdiff_rel_{head}_vs_{f}"] = (float(np.abs(d.data).max()) if d.nnz else 0.0) / scale
    line["stream_copy_GBps"] = stream_copy_gbps(torch)
    line["environment"] = environment(torch, w.seed)
    line["kernel_ms_per_step"] = out[head]["kernel_ms_per_step"]
    line["dense_kernel_avg_ms"] = out[head]["dense_kernel_avg_ms"]
    line["contraction_variant"] = out[head]["contraction_variant"]
    line["trials_per_step"] = out[head]["trials_per_step"]
    line["final_nnz"] = out[head]["final_nnz"]
    if not args.no_cov_context:
        ctx, om_cov = run_cov_context(torch, X32, p, n, w.lam1, w.lam2, args.steps, args.warmup)
        d = om_cov - oms[head]
        ctx[f"final_omega_maxdiff_rel_vs_obs_{head}"] = (
            (float(np.abs(d.data).max()) if d.nnz else 0.0) / float(np.abs(oms[head].data).max()))
        ctx["cov_over_obs"] = ctx["value"] / out[head]["value"]
        line["cov_form_same_problem"] = ctx
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 iteration)")
        X64 = w.X.astype(np.float32).astype(np.float64)
        del w
        line["cpu_baseline"] = cpu_baseline(X64, 0.4, 0.05)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
