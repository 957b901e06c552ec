#!/usr/bin/env python3
"""Benchmark: multi-bandwidth Gaussian summation on one MI355X.

Headline workload: N = M = 1,000,000 monochromatic points for each of
D = 2, 3, 5, 8 (Gaussian mixtures: D=2 four components sigma 0.05, weights
1/N; D=3 eight components sigma U(0.01,0.1), weights 1/N; D=5 64 components
with sizes ~ k^-1.5, sigma U(0.005,0.05), weights U(0.5,1.5); D=8 16
components sigma 0.1, weights U(0.5,1.5)), 64 bandwidths log-spaced 1e-3..1,
eps = 0.01.  One step is one full gauss_sum call per set (tree build,
moments, traversal, base cases, expansions, post-pass over the whole
bandwidth sweep), inputs resident in device memory: 4 x 6.4e13 point-pair
evaluations per step.

Metric: pair-evals/s equivalent = sum over the sets of M N n_h / (time per
step).  Beside it: the plain GPU exhaustive path on the same sets (one step),
the roofline of the dominant kernel (the base-case tiles; HIP events on the
library's stream over the timed steps), the D=3, 10^5-point, 10-bandwidth
workload with the paper's other dual-tree variants (DFTO, DFDO, DFD), node
bounds, pair order, LSCV and the learned pair policy, and the CPU oracle's
rate on a bounded sample of the headline sets (its exhaustive sum, and its
dual-tree in both traversal modes on a 2,000-point draw).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures (one GPU): FP32 vector peak (packed), clock, CUs.
FP32_PEAK_TFLOPS = 157.3
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
# Non-packed FP32 issue: one VALU instruction per lane per clock per SIMD lane.
LANE_SLOTS_PER_S = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_HZ   # 3.93e13
# Issue cost of one v_exp_f32 in VALU slots, relative to an FMA, measured on
# gfx950 in the tiles' mix (one exp2 beside one multiply and two FMAs: 1.65;
# alone it runs at half the FMA rate).
EXP_SLOTS = 1.65

HEADLINE_DIMS = (2, 3, 5, 8)


def method_flops(D, dist_evals, pair_evals):
    """Algorithmic FP32 work of Gaussian-sum tiles: 3D flops per squared
    distance (D differences, D products, D additions) and 4 per point-pair
    kernel evaluation (scale the exponent, exp2, multiply-add the weighted
    term)."""
    return 3.0 * D * dist_evals + 4.0 * pair_evals


def issue_slots(D, dist_evals, pair_evals, dist_slots_per_dim=2.0):
    """Non-packed VALU issue slots of the same work: dist_slots_per_dim per
    dimension of each squared distance formed on the VALU (difference + FMA; 4
    for the split-float exhaustive tiles; distances from the matrix cores take
    none), and per kernel evaluation one multiply or FMA (exponent), one exp2
    (EXP_SLOTS) and one FMA (accumulation)."""
    return dist_slots_per_dim * D * dist_evals + (2.0 + EXP_SLOTS) * pair_evals


def measured_traffic(kernel_source, profile, kernel):
    """HBM bytes per launch of `kernel` recorded by a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if the kernel source still hashes to the
    recorded prefix (None otherwise: the counters describe an older kernel)."""
    try:
        text = open(profile).read()
        src = open(kernel_source, "rb").read()
    except OSError:
        return None
    m = re.search(r"sha256 prefix: (\w+)", text)
    t = re.search(r"traffic_bytes_per_launch %s = (\d+)" % re.escape(kernel), text)
    if not m or not t or hashlib.sha256(src).hexdigest()[:16] != m.group(1):
        return None
    return float(t.group(1))


def cpu_baseline(sets, n_queries_per_set, seed=0):
    """The FP64 exhaustive oracle on a bounded sample of the sets' queries (all
    references, all bandwidths), single-threaded."""
    from threadpoolctl import threadpool_limits

    from oracle.exhaustive import gauss_sum_exhaustive
    rng = np.random.default_rng(seed)
    evals, t = 0.0, 0.0
    with threadpool_limits(limits=1):
        for wl in sets:
            idx = rng.choice(wl.queries.shape[0], size=n_queries_per_set, replace=False)
            t0 = time.perf_counter()
            gauss_sum_exhaustive(wl.queries[idx], wl.refs, wl.weights, wl.bandwidths)
            t += time.perf_counter() - t0
            evals += float(n_queries_per_set) * wl.refs.shape[0] * len(wl.bandwidths)
    return {"value": evals / t, "unit": "pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 exhaustive oracle, %d random queries of each of %s x all references x "
                      "all bandwidths (%.3g pair-evals in %.1f s)"
                      % (n_queries_per_set, ", ".join(w.name for w in sets), evals, t)}


def cpu_dualtree_baseline(workload_fn, D=3, scale=0.002, leaf=64):
    """The oracle's own dual-tree (FP64, one core) on a small draw of the
    headline recipe, in its frontier mode (the library's schedule) and its
    paper mode (the depth-first recursion of Figures 1 and 7): time per call
    and pair-evals/s equivalent.  A draw this small is all the pure-Python
    traversal finishes in seconds, so its rate says nothing about 10^6 points."""
    from threadpoolctl import threadpool_limits

    from oracle.dualtree import dualtree
    wl = workload_fn(4, D=D, scale=scale)
    n = wl.refs.shape[0]
    out = {}
    with threadpool_limits(limits=1):
        for mode in ("level", "depth_first"):
            t0 = time.perf_counter()
            dualtree(wl.refs, wl.refs, wl.weights, wl.bandwidths, wl.eps, leaf_size=leaf, traversal=mode)
            t = time.perf_counter() - t0
            out["frontier" if mode == "level" else "paper"] = {
                "value": float(n) * n * len(wl.bandwidths) / t, "unit": "pair-evals/s", "seconds": t}
    out.update({"cores": 1, "kind": "oracle",
                "sample": "oracle dual-tree on %s (another size of the same recipe), leaf %d" % (wl.name, leaf)})
    return out


def log(*parts):
    """Progress on stderr (the JSON result is the only line on stdout)."""
    print("[bench]", *parts, file=sys.stderr, flush=True)


class Set:
    """One workload resident on the device, with its output buffer."""

    def __init__(self, wl, dev, ctx):
        import torch
        self.wl = wl
        self.ctx = ctx          # shared by the sets (one device workspace)
        self.policy = "rule"
        self.params = None      # this set's trained policy parameters
        self.M, self.N, self.D, self.n_h = wl.queries.shape[0], wl.refs.shape[0], wl.D, len(wl.bandwidths)
        self.rd = torch.from_numpy(wl.refs).to(dev)
        self.qd = self.rd if wl.monochromatic else torch.from_numpy(wl.queries).to(dev)
        self.wd = torch.from_numpy(wl.weights).to(dev)
        self.hd = torch.from_numpy(wl.bandwidths).to(dev)
        self.out = torch.empty((self.n_h, self.M), dtype=torch.float64, device=dev)
        self.pair_evals = float(self.M) * self.N * self.n_h

    def call(self, **kw):
        if kw.get("policy") == "learned":
            self.ctx.policy_set_params(self.params)  # host-side; uploaded with the call
        self.ctx.gauss_sum(self.qd, self.rd, self.wd, self.hd, self.wl.eps, out=self.out, **kw)

    def train_policy(self, workload, scale):
        """The learned pair policy of this set's context, trained on the records
        of a smaller draw of the same workload recipe (another draw; logging
        and training are parameter selection, outside every timed region)."""
        tr = workload(4, D=self.D, scale=scale, draw=1)
        t0 = time.perf_counter()
        self.ctx.gauss_sum(tr.refs, tr.refs, tr.weights, tr.bandwidths, tr.eps, leaf_size=256, log_pairs=1,
                           log_explore=0.3)
        rec, _ = self.ctx.policy_log()
        loss = self.ctx.policy_train(rec, steps=1500, batch=4096, seed=1)
        self.params = self.ctx.policy_params()
        self.train_info = {"trained_on": tr.name + " (another draw)", "records": int(rec.shape[0]),
                           "loss": loss, "train_s": time.perf_counter() - t0}


def timed(sets, steps, warmup, opts_of):
    """warmup untimed steps, then `steps` timed steps; a step is one blocking
    gauss_sum call per set.  Returns the step time, per-set times and the
    per-set sums of the base / exhaustive tile timers and work counters."""
    import torch
    for i in range(warmup):
        for s in sets:
            s.call(**opts_of(s))
            log("warm-up %d %s %s" % (i, s.wl.name, opts_of(s)))
    torch.cuda.synchronize()
    per = [dict(t=0.0, k_ms=np.zeros(12), k_launches=np.zeros(12, dtype=np.int64), base_evals=0,
                dist_evals=0, mfma_evals=0) for _ in sets]
    t0 = time.perf_counter()
    for _ in range(steps):
        for s, acc in zip(sets, per):
            ts = time.perf_counter()
            # HIP events around the dominant tiles only (kernel_timing=2):
            # timing every kernel class adds tens of event records per call
            s.call(kernel_timing=2, **opts_of(s))
            acc["t"] += time.perf_counter() - ts
            st = s.ctx.stats()
            acc["k_ms"] += np.array(st.k_ms[:])
            acc["k_launches"] += np.array(st.k_launches[:])
            acc["base_evals"] += st.base_pair_evals
            acc["dist_evals"] += st.base_dist_evals
            acc["mfma_evals"] += st.base_mfma_pair_evals
            acc["leaf"], acc["method"] = st.tuned_leaf_size, st.tuned_method
        log("step %s: %s" % (opts_of(sets[0]), ", ".join("%s %.1f ms" % (s.wl.name, a["t"] * 1e3)
                                                            for s, a in zip(sets, per))))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / max(1, steps)
    for acc in per:
        acc["t"] /= max(1, steps)
    return t, per


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", default=",".join(str(d) for d in HEADLINE_DIMS),
                    help="dimensions of the headline sets (10^6 points, 64 bandwidths each)")
    ap.add_argument("--cpu-queries", type=int, default=12, help="oracle sample: queries per headline set")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exhaustive", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the D=3, 10^5-point workload and its variant legs")
    ap.add_argument("--no-variants", action="store_true", help="skip the DFTO, DFDO, DFD and LSCV legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-policy leg")
    ap.add_argument("--leg-steps", type=int, default=10, help="timed steps of each leg")
    ap.add_argument("--policy", choices=("auto", "rule", "learned"), default="auto",
                    help="pair policy of the headline sets; auto (default): per set the faster of the "
                         "rule and the learned policy, timed once each after the warm-up (the policy "
                         "is trained on a 5%% draw of the set's recipe; untimed parameter selection)")
    ap.add_argument("--leaf-size", type=int, default=0,
                    help="kd-tree leaf size; 0 (default): chosen by the library's autotuner "
                         "during the warm-up steps")
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

    dev = torch.device("cuda:0")
    dims = [int(x) for x in args.dims.split(",") if x]
    ctx = g.Context(0)
    sets = [Set(workload(4, D=D), dev, ctx) for D in dims]
    tune = dict(leaf_size=args.leaf_size) if args.leaf_size > 0 else dict(autotune=1)

    if args.calib_copy_mib > 0:
        xc = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        yc = torch.empty_like(xc)
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc

    # ---- parameter selection (untimed): leaf size by the library's autotuner,
    # then, per set, the pair policy
    policy_ab = {}
    for s in sets:
        s.call(method="dualtree", **tune)
        s.leaf = s.ctx.stats().tuned_leaf_size
        s.method = s.ctx.stats().tuned_method
        log("tuned %s: method %d leaf %d" % (s.wl.name, s.method, s.leaf))
        if args.policy == "rule" or s.method != g.GS_DUALTREE:
            continue
        s.train_policy(workload, 0.05)
        if args.policy == "learned":
            s.policy = "learned"
            continue
        t = {}
        for pol in ("rule", "learned", "rule", "learned"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.call(method="dualtree", leaf_size=s.leaf, policy=pol)
            torch.cuda.synchronize()
            t[pol] = min(t.get(pol, 1e30), time.perf_counter() - t0)
        s.policy = "learned" if t["learned"] < t["rule"] else "rule"
        policy_ab[s.wl.name] = {"rule_ms": t["rule"] * 1e3, "learned_ms": t["learned"] * 1e3,
                                "speedup_vs_rule": t["rule"] / t["learned"], **s.train_info}
        log("policy %s: rule %.1f ms, learned %.1f ms -> %s" % (s.wl.name, t["rule"] * 1e3, t["learned"] * 1e3,
                                                               s.policy))

    def headline_opts(s):
        if s.method != g.GS_DUALTREE:
            return dict(method="exhaustive")
        return dict(method="dualtree", leaf_size=s.leaf, policy=s.policy)

    # ---- headline: the dual-tree sweep of every set
    t_dt, per = timed(sets, args.steps, args.warmup, headline_opts)
    pair_evals = sum(s.pair_evals for s in sets)
    names = {g.GS_DUALTREE: "dualtree", g.GS_EXHAUSTIVE: "exhaustive"}
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
        "config": {"workload": "d%s_n1000000_mono_64h" % "".join(str(d) for d in dims),
                   "D": dims, "N": sets[0].N, "M": sets[0].M, "n_bandwidths": sets[0].n_h,
                   "eps": sets[0].wl.eps, "autotune": args.leaf_size <= 0,
                   "method": {s.wl.name: names.get(a["method"], "?") for s, a in zip(sets, per)},
                   "leaf_size": {s.wl.name: int(a["leaf"]) for s, a in zip(sets, per)},
                   "policy": {s.wl.name: s.policy for s in sets},
                   "parallelism": "single-gpu"},
    }
    result["per_set"] = {}
    for s, a in zip(sets, per):
        entry = {"ms_per_step": a["t"] * 1e3, "value": s.pair_evals / a["t"],
                 "base_pair_evals_frac": a["base_evals"] / max(1, args.steps) / s.pair_evals,
                 "base_evals_per_distance": a["base_evals"] / max(1, a["dist_evals"]),
                 "mfma_distance_frac": a["mfma_evals"] / max(1, a["base_evals"])}
        n = a["k_launches"][_lib.K_BASE]
        if n > 0:
            ms = a["k_ms"][_lib.K_BASE]
            entry["base_kernel_ms"] = ms / max(1, args.steps)
            entry["base_tflops"] = method_flops(s.D, a["dist_evals"], a["base_evals"]) / (ms * 1e-3) / 1e12
        result["per_set"][s.wl.name] = entry
    if policy_ab:
        result["policy_ab"] = policy_ab

    # Dominant kernel of the step: the bandwidth-fused base tiles, all sets
    # (HIP events on the library's stream around each launch, timed steps only).
    n_base = sum(int(a["k_launches"][_lib.K_BASE]) for a in per)
    if n_base > 0:
        ms = sum(a["k_ms"][_lib.K_BASE] for a in per)
        flops = sum(method_flops(s.D, a["dist_evals"], a["base_evals"]) for s, a in zip(sets, per))
        # distances on the VALU only for the kernel evaluations the MFMA path did not take
        slots = sum(issue_slots(s.D, a["dist_evals"] * (1.0 - a["mfma_evals"] / max(1, a["base_evals"])),
                                a["base_evals"]) for s, a in zip(sets, per))
        achieved = flops / (ms * 1e-3) / 1e12
        issue_peak = LANE_SLOTS_PER_S * flops / slots / 1e12
        traffic = []
        for s, a in zip(sets, per):
            if a["k_launches"][_lib.K_BASE] == 0:
                continue
            traffic.append(measured_traffic(
                os.path.join(ROOT, "paper_1206_6857_amd", "csrc", "k_base.hip"),
                os.path.join(ROOT, "profiles", "base_fused_kernel_d%s_n1000000_mono_64h_hbm_bytes.txt"
                             % "".join(str(d) for d in dims)),
                "base_fused_kernel<%d>" % s.D))
        result["roofline"] = {
            "bound": "alu", "kernel": "base_fused_kernel", "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": (float(np.mean(traffic)) if traffic and all(x is not None for x in traffic) else None),
            "avg_launch_ms": ms / n_base,
            "work_per_launch": {"pair_evals": sum(a["base_evals"] for a in per) / n_base,
                                "dist_evals": sum(a["dist_evals"] for a in per) / n_base,
                                "flops": flops / n_base},
            "issue_model": {"peak_tflops": issue_peak, "frac": achieved / issue_peak,
                            "note": "non-packed FP32 issue (3.93e13 lane-slots/s) at this kernel's "
                                    "mix: 2D slots per distance formed on the VALU (none for the "
                                    "distances the MFMA path forms), 2 + %g per kernel evaluation"
                                    % EXP_SLOTS}}

    # ---- the plain GPU exhaustive path on the same sets (one step: ~20 s per set)
    if not args.no_exhaustive:
        t_ex, per_ex = timed(sets, 1, 0, lambda s: dict(method="exhaustive"))
        ex = {"value": pair_evals / t_ex, "ms_per_step": t_ex * 1e3, "steps": 1}
        ms = sum(a["k_ms"][_lib.K_EXHAUSTIVE] for a in per_ex)
        if ms > 0:
            # one squared distance per point pair and block of up to 16 bandwidths
            flops = sum(method_flops(s.D, float(s.M) * s.N * -(-s.n_h // 16), s.pair_evals) for s in sets)
            slots = sum(issue_slots(s.D, float(s.M) * s.N * -(-s.n_h // 16), s.pair_evals, 4.0) for s in sets)
            ach = flops / (ms * 1e-3) / 1e12
            ex["roofline"] = {"bound": "alu", "kernel": "exhaustive_kernel", "achieved": ach,
                              "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                              "issue_model": {"peak_tflops": LANE_SLOTS_PER_S * flops / slots / 1e12,
                                              "frac": ach / (LANE_SLOTS_PER_S * flops / slots / 1e12)}}
        ex["per_set_ms"] = {s.wl.name: a["t"] * 1e3 for s, a in zip(sets, per_ex)}
        result["exhaustive"] = ex
        result["dualtree_over_exhaustive"] = t_ex / t_dt

    # ---- the D=3, 10^5-point, 10-bandwidth workload and the paper's variants on it
    if not args.no_legs:
        small = Set(workload(1), dev, ctx)
        ls = args.leg_steps
        t1, p1 = timed([small], ls, 1, lambda s: dict(method="dualtree", **tune))
        leaf = int(p1[0]["leaf"])
        leg = {"workload": small.wl.name, "ms_per_step": t1 * 1e3, "value": small.pair_evals / t1,
               "leaf_size": leaf, "method": names.get(p1[0]["method"], "?"),
               "base_pair_evals_frac": p1[0]["base_evals"] / ls / small.pair_evals}
        pc = ctx.pair_counts(small.n_h)
        leg["pairs"] = {k: int(pc[:, i].sum()) for i, k in enumerate(["FD", "DH", "DL", "H2L", "BASE", "SPLIT"])}
        if p1[0]["method"] == g.GS_DUALTREE:
            fixed = dict(leaf_size=leaf, autotune=0)
            t_sr, p_sr = timed([small], ls, 1, lambda s: dict(method="dualtree", node_bounds="sphere_rect",
                                                                      **fixed))
            leg["sphere_rect_bounds"] = {"ms_per_step": t_sr * 1e3, "speedup_vs_box": t1 / t_sr,
                                         "base_pair_evals_frac": p_sr[0]["base_evals"] / ls / small.pair_evals}
            # best-first walk of every query node's list (decreasing dmin^2)
            t_ff, p_ff = timed([small], ls, 1, lambda s: dict(method="dualtree", pair_order="far_first", **fixed))
            leg["far_first_order"] = {"ms_per_step": t_ff * 1e3, "speedup_vs_tree": t1 / t_ff,
                                      "base_pair_evals_frac": p_ff[0]["base_evals"] / ls / small.pair_evals}
            if not args.no_variants:
                variants = {}
                for m in ("dfto", "dfdo", "dfd"):
                    t_m, p_m = timed([small], ls, 1, lambda s, m=m: dict(method=m, **fixed))
                    pc_m = ctx.pair_counts(small.n_h)
                    variants[m] = {"ms_per_step": t_m * 1e3, "time_vs_dito": t_m / t1,
                                   "pairs": {k: int(pc_m[:, i].sum())
                                             for i, k in enumerate(["FD", "DH", "DL", "H2L", "BASE", "SPLIT"])},
                                   "base_pair_evals_frac": p_m[0]["base_evals"] / ls / small.pair_evals}
                leg["variants"] = variants
                # bandwidth selection (least-squares cross-validation): one sweep
                # over h and sqrt(2) h plus the score reduction
                ctx.lscv(small.rd, small.hd, small.wl.eps, leaf_size=leaf)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(ls):
                    scores, bounds = ctx.lscv(small.rd, small.hd, small.wl.eps, leaf_size=leaf)
                torch.cuda.synchronize()
                t_cv = (time.perf_counter() - t0) / ls
                k = int(np.argmin(scores))
                leg["lscv"] = {"ms_per_call": t_cv * 1e3, "h_min": float(small.wl.bandwidths[k]),
                               "score_bound_max": float(np.max(bounds))}
            if not args.no_learned:
                # the learned pair policy, trained on another draw of the same
                # workload (logging and training are parameter selection, untimed)
                tr = workload(1, draw=1)
                t0 = time.perf_counter()
                ctx.gauss_sum(tr.refs, tr.refs, tr.weights, tr.bandwidths, tr.eps, leaf_size=leaf, log_pairs=1,
                              log_explore=0.3)
                rec, _ = ctx.policy_log()
                loss = ctx.policy_train(rec, steps=1500, batch=4096, seed=1)
                small.params = ctx.policy_params()
                t_train = time.perf_counter() - t0
                t_lp, _ = timed([small], ls, 1, lambda s: dict(method="dualtree", policy="learned", **fixed))
                st_lp = ctx.stats()
                leg["learned_policy"] = {
                    "ms_per_step": t_lp * 1e3, "speedup_vs_rule": t1 / t_lp,
                    "train_records": int(rec.shape[0]), "train_loss": loss, "train_s": t_train,
                    "policy_calls": int(st_lp.policy_calls), "policy_overrides": int(st_lp.policy_overrides),
                    "trained_on": tr.name + " (another draw)"}
        if not args.no_exhaustive:
            t_e1, _ = timed([small], ls, 1, lambda s: dict(method="exhaustive"))
            leg["exhaustive_ms_per_step"] = t_e1 * 1e3
            leg["dualtree_over_exhaustive"] = t_e1 / t1
        result["legs"] = {small.wl.name: leg}
        del small

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline([s.wl for s in sets], args.cpu_queries)
        result["cpu_baseline"]["dualtree"] = cpu_dualtree_baseline(workload)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
