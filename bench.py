#!/usr/bin/env python
"""Block Vecchia benchmark on one MI355X.

A step is one evaluation of the block Vecchia log-likelihood together with
its adjoint gradient w.r.t. (sigma2, range, nugget), in the FP32-bulk
precision (FP64 accumulation, FP64 re-factorisation of guard-flagged blocks),
on the 1e6-point 3-D workload: x, y uniform in [0,1], z uniform in [0,0.2],
Matern nu = 2.5, sigma2 = 1, ranges 0.05/0.05/0.01, nugget 1e-3, y drawn by the
sequential Vecchia simulator with 150 neighbours, 50,000 K-means blocks in
random order, 120 neighbours per block.  Inputs are resident in HBM before
the timed region; preprocessing (simulation, K-means, neighbours, plan) is
untimed.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-Vecchia loglik evals/s and points/s at n=1e6, FP32 vs FP64 @1e-4 rel err"
FP32_PEAK = 157.3e12   # MI355X published FP32 peak (vector and dense matrix) FLOP/s
FP64_PEAK = 78.6e12


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("wave_kernel.hpp", "bv_wave_f32.hip", "bv_wave_f64.hip", "bv_mfma.hip", "bv_adjoint.hip",
              "bv_forward.hip", "common.hpp", "internal.hpp", "api.hip"):
        with open(os.path.join(ROOT, "paper_2410_04477_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_flops(p, m, l):
    """Algorithmic flops of one block's value + gradient: joint factorisation and
    solves (p^3/3 + p^2), covariance generation (30 flop-equivalents per lower-
    triangle entry) and the adjoint's extra work (3 m^2 l + 2 m^2)."""
    return p ** 3 / 3.0 + p ** 2 + 30.0 * p * (p + 1) / 2.0 + 3.0 * m * m * l + 2.0 * m * m


def value_flops(p):
    """Algorithmic flops of one block's value: joint factorisation and solves
    (p^3/3 + p^2) and covariance generation (30 per lower-triangle entry)."""
    return p ** 3 / 3.0 + p ** 2 + 30.0 * p * (p + 1) / 2.0


def span_roofline(kt, nclasses, flops, peak, kernel):
    """Roofline over the span of one call's concurrent size-class launches
    (HIP events on the class streams), averaged over the timed calls."""
    span_ms, span_n = kt[nclasses]
    span_s = span_ms / span_n / 1e3
    return {"bound": "mfma", "achieved": flops / span_s / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": flops / span_s / peak, "kernel": kernel, "avg_launch_ms": span_s * 1e3,
            "flops_per_launch": flops}


def simulate_field(w, locs, locs_new, dev):
    """y at the n observed locations (returned in their original order) and at
    the held-out ones, by the sequential Vecchia simulator with w.sim_m
    neighbours: the observed points in a seeded random order, then the
    held-out points."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2410_04477_amd import api

    th0 = w.theta
    n_new = locs_new.shape[0]
    order = W.point_permutation(w.n, w.seed_y)
    inv_order = np.argsort(order)
    metric = list(w.metric_scale)
    locs_ord = torch.tensor(np.vstack([locs[order], locs_new]), device=dev)
    unit = torch.arange(w.n + n_new + 1, dtype=torch.int32, device=dev)
    log(f"simulating y: n={w.n} (+{n_new} held out), {w.sim_m} neighbours")
    snptr, snidx = api.neighbors(locs_ord, unit, w.sim_m, metric)
    z = torch.tensor(np.concatenate([W.standard_normal(w.n, w.seed_y), W.standard_normal(n_new, w.seed_y + 1)]),
                     device=dev)
    y_ord = api.simulate(locs_ord, snptr, snidx, (th0.sigma2, th0.beta, th0.nugget, th0.nu, th0.aniso), z)
    y = api.permute_rows(y_ord[:w.n].contiguous(), torch.tensor(inv_order, device=dev))
    y_new = y_ord[w.n:].contiguous()
    torch.cuda.synchronize()
    return y, y_new



def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--engine", default="mfma", choices=["mfma", "mfma_wg", "tiles"])
    ap.add_argument("--scale", type=int, default=1,
                    help="multiply the workload's n and block count (same points per block and m)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-prediction", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration under rocprofv3)")
    ap.add_argument("--print-sha", action="store_true", help="print the kernel source hash and exit")
    args = ap.parse_args()
    if args.print_sha:
        print(kernel_source_sha())
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads as W
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd.model import BlockVecchia

    w = W.WORKLOADS[args.workload]
    if args.scale != 1:
        w = W.scaled(w, w.n * args.scale, tag=f"x{args.scale}")
    dev = torch.device("cuda:0")
    th0 = w.theta
    t_setup = time.perf_counter()

    # ---- synthetic data: sequential Vecchia draw (sim_m neighbours) ----------
    # n_new held-out locations are drawn after the n observed ones in the
    # simulation order, so the observed values do not depend on them
    locs = W.locations(w)
    n_new = 0 if args.no_prediction else w.n // 10
    locs_new = W.new_locations(w, n_new)
    metric = list(w.metric_scale)
    y, y_new = simulate_field(w, locs, locs_new, dev)
    t_sim = time.perf_counter() - t_setup

    # ---- preprocessing: K-means blocks, random order, neighbours, plan -------
    log(f"preprocessing: bc={w.bc}, m={w.m}")
    t1 = time.perf_counter()
    model = BlockVecchia(locs, y, w.bc, w.m, th0.nu, W.kmeans_init(w.n, w.bc, w.seed_kmeans),
                         W.block_permutation(w.bc, w.seed_kmeans), th0.aniso[: w.d], w.kmeans_iters,
                         engine=args.engine)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t1
    plan = model.plan
    thetas = [model.theta(t.sigma2, t.beta, t.nugget) for t in W.theta_cycle_c3(w)]
    log(f"setup done: simulate {t_sim:.1f}s, preprocess {t_pre:.1f}s, kmeans iters {model.kmeans_iters}, "
        f"buckets {plan.buckets()}")

    def run(precision: str, grad: bool, k: int) -> None:
        for i in range(k):
            th = [thetas[i % len(thetas)]]
            if grad:
                model.loglik_grad(th, precision)
            else:
                model.loglik(th, precision)

    def timed(precision: str, grad: bool, k: int, warm: int, with_timing: bool = False):
        run(precision, grad, warm)
        torch.cuda.synchronize()
        if with_timing:
            plan.set_timing(True)
            plan.timing(reset=True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        run(precision, grad, k)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = plan.timing(reset=True) if with_timing else None
        if with_timing:
            plan.set_timing(False)
        return wall, ev0.elapsed_time(ev1) / 1e3, kt

    # ---- headline: FP32-bulk value + gradient --------------------------------
    log(f"timing fp32-bulk loglik+grad: warmup {args.warmup}, steps {args.steps}")
    wall, gpu_s, kt = timed("fp32", True, args.steps, args.warmup, with_timing=True)
    ms_step = 1e3 * wall / args.steps
    evals = args.steps / wall

    # ---- roofline of the dominant kernel (live HIP events) -------------------
    bp = plan.block_ptr.cpu().numpy().astype(np.int64)
    npt = plan.nbr_ptr.cpu().numpy().astype(np.int64)
    lsz, msz = np.diff(bp), np.diff(npt)
    psz = lsz + msz
    sched = plan.schedule().cpu().numpy()
    # the size classes run concurrently on the plan's streams: the roofline is
    # taken over their common span (first class launch to last), per call
    classes = plan.buckets()
    span_ms, span_n = kt[len(classes)]
    avg_span_s = span_ms / span_n / 1e3
    names, cls = [], []
    flops_launch = 0.0
    for q, (cfg, nb) in enumerate(classes):
        off0, off1 = int(plan.c.bucket_off[q]), int(plan.c.bucket_off[q + 1])
        blk = sched[off0:off1]
        fq = float(np.sum(step_flops(psz[blk].astype(np.float64), msz[blk].astype(np.float64),
                                     lsz[blk].astype(np.float64))))
        flops_launch += fq
        kn = plan.class_kernel(q, "fp32", True)
        names.append(kn)
        cls.append({"kernel": kn, "blocks": int(nb), "flops": fq, "ms_per_step": kt[q][0] / args.steps})
    achieved = flops_launch / avg_span_s
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tr = json.load(fh)
        # the counters were taken on the default workload: other sizes report none
        if (args.workload == "C3" and args.scale == 1 and tr.get("kernel_source_sha") == kernel_source_sha()
                and all(n in tr for n in names)):
            traffic = float(sum(tr[n]["bytes_per_launch"] for n in names))
    roofline = {"bound": "alu" if plan.engine == "tiles" else "mfma", "achieved": achieved / 1e12,
                "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK, "traffic": traffic,
                "kernel": f"{len(names)} concurrent size classes ({', '.join(names)})",
                "launch": "span of one call's concurrent size-class launches (first start to last end)",
                "avg_launch_ms": avg_span_s * 1e3, "flops_per_launch": flops_launch,
                "blocks_per_launch": int(sum(c["blocks"] for c in cls)),
                "share_of_step": avg_span_s / (gpu_s / args.steps) if gpu_s > 0 else None,
                "size_classes": cls}
    total_flops_step = float(np.sum(step_flops(psz.astype(np.float64), msz.astype(np.float64),
                                               lsz.astype(np.float64))))

    # ---- variants and accuracy ----------------------------------------------
    variants = {}
    flops_value = float(np.sum(value_flops(psz.astype(np.float64))))
    if not args.no_variants:
        k2 = max(3, args.steps // 2)
        for prec, grad in (("fp64", True), ("fp64", False), ("fp32", False)):
            log(f"timing {prec} {'loglik+grad' if grad else 'loglik'}")
            wv, _, ktv = timed(prec, grad, k2, 1, with_timing=True)
            key = f"{prec}_{'loglik_grad' if grad else 'loglik'}"
            variants[f"{key}_evals_per_s"] = k2 / wv
            vnames = [plan.class_kernel(q, prec, grad) for q in range(len(classes))]
            variants[f"{key}_roofline"] = span_roofline(
                ktv, len(classes), flops_launch if grad else flops_value, FP64_PEAK if prec == "fp64" else FP32_PEAK,
                f"{len(classes)} concurrent size classes ({', '.join(vnames)})")
        variants["fp32_loglik_grad_evals_per_s"] = evals
        variants["speedup_fp32_over_fp64_loglik_grad"] = evals / variants["fp64_loglik_grad_evals_per_s"]
        variants["speedup_fp32_over_fp64_loglik"] = (variants["fp32_loglik_evals_per_s"]
                                                     / variants["fp64_loglik_evals_per_s"])
        # an order outside the closed forms (Bessel-form kernels), same workload
        log("timing fp32 loglik+grad at nu = 1.0 (Bessel form)")
        th_g = [(t[0], t[1], t[2], 1.0, t[4]) for t in thetas]
        for th in th_g[:1]:
            model.loglik_grad([th], "fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k2):
            model.loglik_grad([th_g[i % len(th_g)]], "fp32")
        torch.cuda.synchronize()
        variants["fp32_loglik_grad_nu1.0_bessel_evals_per_s"] = k2 / (time.perf_counter() - t0)
        # value and all four derivatives (sigma2, range, nugget, nu) from the adjoint
        log("timing fp32 loglik + gradient incl. d / d nu at nu = 1.0 (adjoint)")
        model.loglik_grad_nu(th_g[:1], "fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k2):
            model.loglik_grad_nu([th_g[i % len(th_g)]], "fp32")
        torch.cuda.synchronize()
        variants["fp32_loglik_grad_with_nu_nu1.0_evals_per_s"] = k2 / (time.perf_counter() - t0)
        # d l / d nu alone as a central difference (two FP64 Bessel-form log-likelihoods per theta)
        log("timing d l / d nu at nu = 1.0 (central difference)")
        model.loglik_dnu(th_g[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k2):
            model.loglik_dnu([th_g[i % len(th_g)]])
        torch.cuda.synchronize()
        variants["fp64_loglik_dnu_nu1.0_evals_per_s"] = k2 / (time.perf_counter() - t0)
    tt = [thetas[0]]
    l64, g64, _, _, gp64 = model.loglik_grad(tt, "fp64", want_partial=True)
    l32, g32, c32, _, _ = model.loglik_grad(tt, "fp32")
    l64, l32 = float(l64[0]), float(l32[0])
    g64n, g32n = g64[0].cpu().numpy(), g32[0].cpu().numpy()
    # the gradient is a sum of per-block terms that largely cancel near the
    # generating theta; its error is also stated against sum_i |dl_i|
    gscale = gp64[0].abs().sum(0).cpu().numpy()
    accuracy = {"loglik_fp64": l64, "loglik_fp32": l32, "rel_err_loglik_fp32_vs_fp64": abs(l32 - l64) / abs(l64),
                "rel_err_grad_fp32_vs_fp64": float(np.linalg.norm(g32n - g64n) / np.linalg.norm(g64n)),
                "grad_err_per_component_vs_sum_abs_block_terms": [float(v) for v in np.abs(g32n - g64n) / gscale],
                "fp32_blocks_refactored": int(c32[0, 0]), "blocks": int(plan.bc)}

    # ---- prediction (Alg. 2) and conditional simulation at the held-out points --
    prediction = None
    if n_new > 0:
        prediction = bench_prediction(model, locs_new, y_new, w, th0, metric, args.steps, dev)

    # ---- blocks above the one-wave limit: the accuracy study's BV-1500-450 ----
    large_blocks = None
    if not args.no_prediction and args.scale == 1:
        large_blocks = bench_large_blocks(W.C5, max(3, args.steps // 2), dev)

    # ---- block orderings (preprocessing, untimed in the step): Morton, Hilbert, KD-tree, maxmin --
    t_order = {}
    if not args.no_prediction:
        for method in ("morton", "hilbert", "kdtree", "maxmin"):
            log(f"reordering {plan.bc} blocks: {method}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.reorder_blocks(model.locs_perm, plan.block_ptr, method, metric)
            torch.cuda.synchronize()
            t_order[f"reorder_{method}"] = time.perf_counter() - t0

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same blocks --
    cpu = None
    if not args.no_cpu_baseline:
        cpu, sample, o_l, o_g = cpu_baseline(model, plan, bp, npt, th0, args.cpu_seconds)
        accuracy["vs_oracle"] = accuracy_vs_oracle(model, th0, sample, o_l, o_g)

    out = {
        "metric": METRIC,
        "value": evals,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={w.n} {w.d}-D, nu={th0.nu}, sigma2={th0.sigma2}, "
                               f"ranges {[th0.beta * a for a in th0.aniso[:w.d]]}, nugget={th0.nugget}, "
                               f"bc={w.bc}, m={w.m}, y by sequential Vecchia ({w.sim_m} nbrs)",
                   "step": "loglik + adjoint gradient (sigma2, range, nugget)",
                   "precision": "fp32-bulk, fp64 accumulation and guard re-factorisation",
                   "n": w.n, "bc": int(plan.bc), "m": w.m, "engine": args.engine},
        "points_per_s": evals * w.n,
        "gflops_per_step": total_flops_step / 1e9,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "accuracy": accuracy,
        "setup_s": {"simulate": t_sim, "preprocess": t_pre, **t_order},
        "prediction": prediction,
        "large_blocks": large_blocks,
    }
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * 8
    print(json.dumps(out), flush=True)
    return 0


def pred_flops(m, l):
    """Algorithmic flops of one prediction block: Cholesky of the neighbour
    covariance (m^3/3), the triangular solves of K_NB and y_N (m^2 (l + 1)),
    the Schur update (m (l + 1)^2) and covariance generation (30 per entry)."""
    p = m + l
    return m ** 3 / 3.0 + m * m * (l + 1) + m * (l + 1) ** 2 + 30.0 * p * (p + 1) / 2.0


def bench_large_blocks(w, steps, dev):
    """Log-likelihood (value) on a workload whose blocks exceed the one-wave
    limit (m_i + l_i > 175): the bordered matrix of each block is generated
    into a workspace slot and factored left-looking in 16-column panels.
    FP64 and FP32-bulk; the roofline is the large-block launch alone, from
    the plan's own HIP events on the stream it runs on."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2410_04477_amd.model import BlockVecchia

    th0 = w.theta
    locs = W.locations(w)
    y, _ = simulate_field(w, locs, np.zeros((0, w.d)), dev)
    t0 = time.perf_counter()
    model = BlockVecchia(locs, y, w.bc, w.m, th0.nu, W.kmeans_init(w.n, w.bc, w.seed_kmeans),
                         W.block_permutation(w.bc, w.seed_kmeans), th0.aniso[: w.d], w.kmeans_iters)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    plan = model.plan
    classes = plan.buckets()
    ql = [q for q in range(len(classes)) if plan.class_kernel(q, "fp64", False).startswith("bv_large_kernel")]
    assert len(ql) == 1 and int(plan.c.nlarge) > 0, "the workload has no blocks above the one-wave limit"
    ql = ql[0]
    sched = plan.schedule().cpu().numpy()
    bp = plan.block_ptr.cpu().numpy().astype(np.int64)
    npt = plan.nbr_ptr.cpu().numpy().astype(np.int64)
    psz = (np.diff(bp) + np.diff(npt)).astype(np.float64)
    blk = sched[int(plan.c.bucket_off[ql]):int(plan.c.bucket_off[ql + 1])]
    flops_large = float(np.sum(value_flops(psz[blk])))
    thetas = [model.theta(t.sigma2, t.beta, t.nugget) for t in W.theta_cycle_c3(w)]
    out = {"workload": f"{w.name}: n={w.n} 2-D uniform, nu={th0.nu}, sigma2={th0.sigma2}, beta={th0.beta}, "
                       f"nugget={th0.nugget}, bc={w.bc}, m={w.m}, random block order, y by sequential "
                       f"Vecchia ({w.sim_m} nbrs)",
           "n": w.n, "bc": int(plan.bc), "m": w.m, "large_blocks": int(plan.c.nlarge),
           "p_max": int(psz.max()), "p_mean_large": float(psz[blk].mean()), "preprocess_s": t_pre}
    for prec in ("fp64", "fp32"):
        for i in range(2):
            model.loglik([thetas[i % len(thetas)]], prec)
        torch.cuda.synchronize()
        plan.set_timing(True)
        plan.timing(reset=True)
        t0 = time.perf_counter()
        for i in range(steps):
            _, cnt = model.loglik([thetas[i % len(thetas)]], prec)[:2]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        kt = plan.timing(reset=True)
        plan.set_timing(False)
        k_s = kt[ql][0] / kt[ql][1] / 1e3
        peak = FP64_PEAK if prec == "fp64" else FP32_PEAK
        kname = plan.class_kernel(ql, prec, False)
        out[prec] = {"loglik_evals_per_s": 1.0 / wall, "ms": wall * 1e3,
                     "roofline": {"bound": "mfma", "achieved": flops_large / k_s / 1e12, "peak": peak / 1e12,
                                  "unit": "TFLOP/s", "frac": flops_large / k_s / peak, "kernel": kname,
                                  "avg_launch_ms": k_s * 1e3, "flops_per_launch": flops_large,
                                  "share_of_step": k_s / wall},
                     "blocks_refactored_fp64": int(cnt[0, 0]) if prec == "fp32" else 0}
    l64 = float(model.loglik([thetas[0]], "fp64")[0][0])
    l32 = float(model.loglik([thetas[0]], "fp32")[0][0])
    out["rel_err_loglik_fp32_vs_fp64"] = abs(l32 - l64) / abs(l64)
    return out


def bench_prediction(model, locs_new, y_new, w, th0, metric, steps, dev):
    """Block Vecchia prediction at n_new held-out points of the same field
    (blocks of about 10 new points, the workload's m observed neighbours each),
    then 1,000 rounds of univariate conditional simulation with PICP and MSPE."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2410_04477_amd import api

    n_new = locs_new.shape[0]
    bc = n_new // 10
    t0 = time.perf_counter()
    ln = torch.tensor(locs_new, device=dev)
    perm, bp, _ = api.blocks(ln, bc, torch.tensor(W.kmeans_init(n_new, bc, w.seed_kmeans + 7), device=dev),
                             torch.tensor(W.block_permutation(bc, w.seed_kmeans + 7), device=dev), metric)
    ln = api.permute_rows(ln, perm)
    yt = api.permute_rows(y_new, perm)
    npt, nid = api.pred_neighbors(model.locs_perm, ln, bp, w.m, metric)
    plan = api.Plan(bp, npt, n_new, 1, "mfma", predict=True)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    th = (th0.sigma2, th0.beta, th0.nugget, th0.nu, th0.aniso)
    for _ in range(2):
        api.predict(plan, model.locs_perm, model.y_perm, ln, nid, th)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        mean, var, _ = api.predict(plan, model.locs_perm, model.y_perm, ln, nid, th)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kt = plan.timing(reset=True)
    plan.set_timing(False)
    nq = int(plan.c.nbuckets)
    span_s = kt[nq][0] / kt[nq][1] / 1e3
    l = np.diff(plan.block_ptr.cpu().numpy()).astype(np.float64)
    m = np.diff(plan.nbr_ptr.cpu().numpy()).astype(np.float64)
    flops = float(np.sum(pred_flops(m, l)))
    gs = [int(plan.c.bucket_cfg[q]) + 1 for q in range(nq)]
    # conditional simulation: the random numbers are drawn on the device (seeded)
    R = 1000
    gen = torch.Generator(device=dev)
    gen.manual_seed(w.seed_y + 2)
    z = torch.randn((R, n_new), generator=gen, dtype=torch.float64, device=dev)
    api.condsim(mean, var, z, yt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        cs = api.condsim(mean, var, z, yt)
    torch.cuda.synchronize()
    t_cs = (time.perf_counter() - t0) / reps
    cs_bytes = R * n_new * 8.0 + 7.0 * n_new * 8   # z once; mean, var, truth in; four outputs
    return {"workload": f"{n_new} held-out points of the same field, {bc} K-means blocks, m={w.m} observed "
                        f"neighbours of {w.n}, FP64",
            "n_new": n_new, "bc": bc, "m": w.m, "ms": wall * 1e3, "points_per_s": n_new / wall,
            "roofline": {"bound": "mfma", "achieved": flops / span_s / 1e12, "peak": FP64_PEAK / 1e12,
                         "unit": "TFLOP/s", "frac": flops / span_s / FP64_PEAK,
                         "kernel": ", ".join(f"bv_wave_kernel<double,{g},4>" for g in gs),
                         "avg_launch_ms": span_s * 1e3, "flops_per_launch": flops},
            "condsim": {"rounds": R, "ms": t_cs * 1e3, "picp": cs["picp"], "mspe": cs["mspe"],
                        "mean_pred_var": float(var.mean()),
                        "roofline": {"bound": "hbm", "achieved": cs_bytes / t_cs / 1e9, "peak": 8000.0,
                                     "unit": "GB/s", "frac": cs_bytes / t_cs / 8e12}},
            "setup_s": t_pre}


def cpu_baseline(model, plan, bp, npt, th0, target_s):
    """FP64 oracle (plain C, OpenMP over blocks) value + gradient on a seeded
    random sample of the workload's blocks, scaled to evaluations per second of
    the whole workload.  Timing only."""
    import numpy as np

    import workloads as W
    from oracle import coracle

    locs = model.locs_perm.cpu().numpy()
    y = model.y_perm.cpu().numpy()
    nidx = model.nbr_idx.cpu().numpy().astype(np.int64)
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    bc = plan.bc
    order = W.rng(12345).permutation(bc)

    def run(S):
        t0 = time.perf_counter()
        vals = coracle.selected_terms(locs, y, bp, npt, nidx, th0, order[:S], with_grad=True, nthreads=cores)
        return time.perf_counter() - t0, vals

    S = min(bc, 1024)     # a pilot large enough that thread start-up does not dominate
    dt, _ = run(S)
    S2 = int(min(bc, max(S, S * target_s / max(dt, 1e-3))))
    dt, (o_l, o_g) = run(S2)
    per_eval = dt * bc / S2
    return ({"value": 1.0 / per_eval, "unit": "evals/s", "cores": cores, "kind": "oracle",
             "sample": f"{S2} of {bc} blocks (seeded random), FP64 loglik + gradient, scaled by {bc}/{S2}",
             "seconds": dt}, order[:S2], o_l, o_g)


def accuracy_vs_oracle(model, th0, sample, o_l, o_g):
    """Per-block terms and gradient rows of the GPU (FP64 and FP32-bulk) at
    the generating theta against the oracle values of the CPU-baseline leg, on
    the blocks that leg evaluated (all of them when its time budget allows).
    The inputs are the benchmark's own (simulated y, library neighbour lists):
    a diagnostic beside the parity tests, which use oracle-side inputs."""
    import numpy as np

    th = [model.theta(th0.sigma2, th0.beta, th0.nugget)]
    out = {"blocks": int(len(sample)), "of": int(model.plan.bc)}
    scale_l = float(np.abs(o_l).sum())
    scale_g = np.abs(o_g).sum(0)
    for prec in ("fp64", "fp32"):
        _, _, cnt, part, gpart = model.loglik_grad(th, prec, want_partial=True)
        pl = part[0].cpu().numpy()[sample]
        pg = gpart[0].cpu().numpy()[sample]
        dl = pl - o_l
        dg = pg - o_g
        out[prec] = {"max_abs_dl_i": float(np.abs(dl).max()),
                     "max_rel_dl_i": float(np.max(np.abs(dl) / np.maximum(np.abs(o_l), 1.0))),
                     "rel_err_sum_l": float(abs(dl.sum()) / abs(o_l.sum())),
                     "sum_abs_dl_over_sum_abs_l": float(np.abs(dl).sum() / scale_l),
                     "grad_rel_err_normwise_rows": float(np.linalg.norm(dg) / np.linalg.norm(o_g)),
                     "grad_err_of_sum_per_component_vs_sum_abs": [float(v) for v in np.abs(dg.sum(0)) / scale_g],
                     "blocks_refactored": int(cnt[0, 0])}
    return out


if __name__ == "__main__":
    sys.exit(main())
