#!/usr/bin/env python3
"""Benchmark: multi-bandwidth Gaussian summation on one MI355X.

Workload (default): D=3, N=M=100,000 monochromatic points from an 8-component
Gaussian mixture (sigma uniform 0.01-0.1), weights 1/N, 10 bandwidths
log-spaced 1e-3..1, eps=0.01.  One step is one full gauss_sum call (tree
build, moments, traversal, base cases, expansions, post-pass) over the whole
bandwidth sweep with inputs already resident in device memory.

Metric: pair-evals/s equivalent = M * N * n_h / (time per step), for the
dual-tree path; the plain GPU exhaustive path is timed beside it.  The JSON
line also carries the roofline of the dominant kernel (HIP-event timing of
that kernel over the timed steps), the paper's other dual-tree variants
(DFTO, DFDO, DFD) on the same workload and leaf size, and the CPU oracle's
rate on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures (one GPU).
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
HBM_BYTES_PER_S = 8.0e12
# Issue cost of one v_exp_f32 in VALU slots (transcendental rate), relative to
# an FMA; measured on gfx950 by the rate probe recorded in the design notes.
EXP_SLOTS = 2.0


def base_tile_model(D):
    """Algorithmic FP32 work of one point-pair kernel evaluation in the
    exhaustive tiles: D subtractions + D FMAs (squared distance), one FMA
    (scaled exponent), one exp2, one FMA (weighted accumulation).
    Returns (flops per pair-eval, VALU issue slots per pair-eval)."""
    flops = D + 2 * D + 2 + 1 + 2
    slots = D + D + 1 + EXP_SLOTS + 1
    return flops, slots


def fused_base_model(D, dist_evals, exp_evals):
    """Algorithmic FP32 work of the bandwidth-fused base tiles: every point pair
    of a regrouped entry forms its squared distance once (D subtractions, D
    FMAs), and each bandwidth of the entry's mask costs one FMA (exponent), one
    exp2 and one FMA (accumulation).  Returns (flops, VALU issue slots)."""
    flops = dist_evals * 3 * D + exp_evals * 5
    slots = dist_evals * 2 * D + exp_evals * (2 + EXP_SLOTS)
    return flops, slots


LANE_SLOTS_PER_S = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_HZ


def alu_peak_pairs_per_s(D):
    return LANE_SLOTS_PER_S / base_tile_model(D)[1]


def measured_traffic(kernel_source, profile):
    """HBM bytes per launch recorded by the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, if the kernel source still hashes to the recorded
    prefix (None otherwise: the counters describe an older kernel)."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        src = open(kernel_source, "rb").read()
    except OSError:
        return None
    m = re.search(r"sha256 prefix: (\w+)", text)
    t = re.search(r"traffic_bytes_per_launch \S+ = (\d+)", text)
    if not m or not t or hashlib.sha256(src).hexdigest()[:16] != m.group(1):
        return None
    return float(t.group(1))


def cpu_baseline(wl, n_queries, seed=0):
    """The FP64 exhaustive oracle on a bounded sample of the workload's queries
    (all references, all bandwidths), single-threaded."""
    from threadpoolctl import threadpool_limits

    from oracle.exhaustive import gauss_sum_exhaustive
    rng = np.random.default_rng(seed)
    idx = rng.choice(wl.queries.shape[0], size=n_queries, replace=False)
    q = wl.queries[idx]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        gauss_sum_exhaustive(q, wl.refs, wl.weights, wl.bandwidths)
        t = time.perf_counter() - t0
    evals = n_queries * wl.refs.shape[0] * len(wl.bandwidths)
    return {"value": evals / t, "unit": "pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 exhaustive oracle, %d of %d queries x all %d references x %d "
                      "bandwidths (%.3g pair-evals in %.1f s)"
                      % (n_queries, wl.queries.shape[0], wl.refs.shape[0], len(wl.bandwidths),
                         evals, t)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=1, help="workload index (see datagen.workload)")
    ap.add_argument("--cpu-queries", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exhaustive", action="store_true")
    ap.add_argument("--leaf-size", type=int, default=0,
                    help="kd-tree leaf size; 0 (default): chosen by the library's autotuner "
                         "during the warm-up steps")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the DFTO, DFDO and DFD legs")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-policy leg (trained on another draw of the workload)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy (y = x * 1) of this many MiB, "
                         "to calibrate HBM byte counters against a known size")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the path runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1206_6857_amd as g
    from paper_1206_6857_amd import _lib
    from paper_1206_6857_amd.datagen import workload

    wl = workload(args.workload)
    M, N, D, n_h = wl.queries.shape[0], wl.refs.shape[0], wl.D, len(wl.bandwidths)
    dev = torch.device("cuda:0")
    rd = torch.from_numpy(wl.refs).to(dev)
    qd = rd if wl.monochromatic else torch.from_numpy(wl.queries).to(dev)
    wd = torch.from_numpy(wl.weights).to(dev)
    hd = torch.from_numpy(wl.bandwidths).to(dev)
    out = torch.empty((n_h, M), dtype=torch.float64, device=dev)
    ctx = g.Context(0)
    pair_evals = float(M) * N * n_h

    tune = dict(leaf_size=args.leaf_size) if args.leaf_size > 0 else dict(autotune=1)

    def run(method, steps, warmup, **extra):
        kw = dict(tune, **extra) if method != "exhaustive" else {}
        for _ in range(max(1, warmup)):
            ctx.gauss_sum(qd, rd, wd, hd, wl.eps, out=out, method=method, **kw)
        torch.cuda.synchronize()
        kms = np.zeros(12)
        kl = np.zeros(12, dtype=np.int64)
        evals = np.zeros(2, dtype=np.int64)
        t0 = time.perf_counter()
        for _ in range(steps):
            # HIP events around the dominant kernel only (kernel_timing=2):
            # timing every kernel class adds tens of event records per call
            ctx.gauss_sum(qd, rd, wd, hd, wl.eps, out=out, method=method, kernel_timing=2, **kw)
            st = ctx.stats()
            kms += np.array(st.k_ms[:])
            kl += np.array(st.k_launches[:])
            evals += (st.base_pair_evals, st.base_dist_evals)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        return t, kms, kl, evals, ctx.stats()

    if args.calib_copy_mib > 0:
        xc = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        yc = torch.empty_like(xc)
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc

    t_dt, kms, kl, evals, st_dt = run("dualtree", args.steps, args.warmup)
    base_evals, dist_evals = int(evals[0]), int(evals[1])
    leaf = st_dt.tuned_leaf_size
    method_used = {g.GS_DUALTREE: "dualtree", g.GS_EXHAUSTIVE: "exhaustive"}.get(st_dt.tuned_method, "?")
    pc = ctx.pair_counts(n_h)
    result = {
        "metric": "pair-evals/sec equiv. at eps=0.01, dual-tree vs GPU exhaustive; % of roofline",
        "value": pair_evals / t_dt,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "D": D, "N": N, "M": M, "n_bandwidths": n_h,
                   "eps": wl.eps, "method": method_used, "leaf_size": leaf,
                   "autotune": args.leaf_size <= 0, "parallelism": "single-gpu"},
    }

    # Dominant kernel of the dual-tree step: the bandwidth-fused base tiles
    # (HIP events on the library's stream around each launch, timed steps only).
    if kl[_lib.K_BASE] > 0:
        n = kl[_lib.K_BASE]
        avg_ms = kms[_lib.K_BASE] / n
        flops, slots = fused_base_model(D, dist_evals / n, base_evals / n)
        achieved = flops / (avg_ms * 1e-3) / 1e12
        peak = LANE_SLOTS_PER_S * flops / slots / 1e12
        traffic = measured_traffic(
            os.path.join(ROOT, "paper_1206_6857_amd", "csrc", "k_base.hip"),
            os.path.join(ROOT, "profiles", "base_fused_kernel_%s_leaf%d_hbm_bytes.txt" % (wl.name, leaf)))
        result["roofline"] = {"bound": "alu", "kernel": "base_fused_kernel", "achieved": achieved,
                              "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                              "traffic": traffic, "avg_launch_ms": avg_ms,
                              "pair_evals_per_launch": base_evals / n,
                              "dist_evals_per_launch": dist_evals / n}
    # Per-class device times from one more call with every class timed
    # (outside the timed region).
    ctx.gauss_sum(qd, rd, wd, hd, wl.eps, out=out, method=method_used, kernel_timing=1, **tune)
    st_k = ctx.stats()
    result["breakdown_ms"] = {
        "stage": st_dt.t_stage_ms, "tree": st_dt.t_tree_ms, "moments": st_dt.t_moments_ms,
        "traverse": st_dt.t_traverse_ms, "work": st_dt.t_work_ms, "post": st_dt.t_post_ms,
        "base_kernel": float(kms[_lib.K_BASE] / args.steps),
        "kernels_one_call": {k: float(st_k.k_ms[i]) for k, i in (
            ("base", _lib.K_BASE), ("decide", _lib.K_DECIDE), ("series", _lib.K_SERIES),
            ("post", _lib.K_POST), ("tree", _lib.K_TREE), ("moments", _lib.K_MOMENTS))}}
    result["pairs"] = {k: int(pc[:, i].sum()) for i, k in enumerate(["FD", "DH", "DL", "H2L", "BASE", "SPLIT"])}
    result["base_pair_evals_frac"] = base_evals / args.steps / pair_evals

    if method_used == "dualtree":
        # Sphere-rectangle node bounds (tighter node-pair distances), same
        # workload and leaf size.
        t_sr, _, _, ev_sr, st_sr = run("dualtree", args.steps, args.warmup, leaf_size=leaf, autotune=0,
                                       node_bounds="sphere_rect")
        pc_sr = ctx.pair_counts(n_h)
        result["sphere_rect_bounds"] = {
            "ms_per_step": t_sr * 1e3, "value": pair_evals / t_sr, "speedup_vs_box": t_dt / t_sr,
            "pairs_decided": int(pc_sr.sum()), "pairs_decided_box": int(pc.sum()),
            "base_pair_evals_frac": int(ev_sr[0]) / args.steps / pair_evals}

    if method_used == "dualtree" and not args.no_variants:
        # The paper's other dual-tree variants on the same workload and leaf
        # size: O(p^D) expansions (DFTO), finite differences with tokens
        # (DFDO) and without (DFD).
        variants = {}
        for m in ("dfto", "dfdo", "dfd"):
            t_m, _, _, ev_m, _ = run(m, args.steps, 1, leaf_size=leaf, autotune=0)
            pc_m = ctx.pair_counts(n_h)
            variants[m] = {"ms_per_step": t_m * 1e3, "value": pair_evals / t_m, "time_vs_dito": t_m / t_dt,
                           "pairs": {k: int(pc_m[:, i].sum())
                                     for i, k in enumerate(["FD", "DH", "DL", "H2L", "BASE", "SPLIT"])},
                           "base_pair_evals_frac": int(ev_m[0]) / args.steps / pair_evals}
        result["variants"] = variants

    if method_used == "dualtree" and not args.no_variants:
        # Bandwidth selection (least-squares cross-validation) over the
        # workload's bandwidths: one sweep over h and sqrt(2) h plus the
        # score reduction, inputs resident on the device.
        for _ in range(max(1, args.warmup)):
            ctx.lscv(rd, hd, wl.eps, leaf_size=leaf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            scores, bounds = ctx.lscv(rd, hd, wl.eps, leaf_size=leaf)
        torch.cuda.synchronize()
        t_cv = (time.perf_counter() - t0) / args.steps
        k = int(np.argmin(scores))
        result["lscv"] = {"ms_per_call": t_cv * 1e3, "bandwidths": n_h, "h_min": float(wl.bandwidths[k]),
                          "score_bound_max": float(np.max(bounds))}

    if not args.no_learned and method_used == "dualtree":
        # The learned pair policy, trained on another draw of the same
        # workload (logging and training are parameter selection, not timed).
        tr = workload(args.workload, draw=1)
        t0 = time.perf_counter()
        ctx.gauss_sum(tr.refs, tr.refs, tr.weights, tr.bandwidths, tr.eps, leaf_size=leaf, log_pairs=1,
                      log_explore=0.3)
        rec, _ = ctx.policy_log()
        loss = ctx.policy_train(rec, steps=1500, batch=4096, seed=1)
        t_train = time.perf_counter() - t0
        t_lp, _, _, _, st_lp = run("dualtree", args.steps, args.warmup, policy="learned")
        result["learned_policy"] = {
            "ms_per_step": t_lp * 1e3, "value": pair_evals / t_lp, "speedup_vs_rule": t_dt / t_lp,
            "train_records": int(rec.shape[0]), "train_loss": loss, "train_s": t_train,
            "policy_calls": int(st_lp.policy_calls), "policy_overrides": int(st_lp.policy_overrides),
            "trained_on": tr.name + " (another draw)"}

    if not args.no_exhaustive:
        t_ex, kms_e, kl_e, _, _ = run("exhaustive", max(1, args.steps), 1)
        ex = {"value": pair_evals / t_ex, "ms_per_step": t_ex * 1e3}
        if kl_e[_lib.K_EXHAUSTIVE] > 0:
            avg_ms = kms_e[_lib.K_EXHAUSTIVE] / kl_e[_lib.K_EXHAUSTIVE]
            ach = pair_evals / (avg_ms * 1e-3)
            ex["roofline"] = {"bound": "alu", "achieved_pair_evals_per_s": ach,
                              "peak_pair_evals_per_s": alu_peak_pairs_per_s(D),
                              "frac": ach / alu_peak_pairs_per_s(D)}
        result["exhaustive"] = ex
        result["dualtree_over_exhaustive"] = t_ex / t_dt

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_queries)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
