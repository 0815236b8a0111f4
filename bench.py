#!/usr/bin/env python3
"""Benchmark of the gravity hot path on one MI355X.

Headline workload (the one the metric names: learned against plain seeding of
the relative criterion): the clustered periodic box of 256^3 = 16 777 216
equal-mass particles drawn with the held-out evaluation seed 2001 (60 % of the
mass in 2000 Hernquist haloes, 40 % uniform), TreePM split r_s = 1.25 L/256
scaled to the mean spacing (mesh 512^3 at 256^3), softening L/(40 * 256), leaf
size 32 (the fastest of 16-40 at this size), p = 3, wavefront groups of 64.

A step is one pass of the whole path: integer mapping -> Morton keys + radix
sort -> octree -> multipoles -> |a| seed -> relative TreePM short-range walk ->
forces in the caller's order.  The seed is the geometric pre-walk (theta =
0.7) for the plain variant and the trained network (features + MLP) for the
learned one.  Inputs are resident in HBM before the timed region.

The metric asks for forces/s at a 99th-percentile relative force error <= 1e-3
against direct summation.  At R_cut = 4.5 r_s the cut-off alone leaves a
99th-percentile error near 0.1 against the untruncated short-range direct
sum, so the walk runs at R_cut = 7 r_s (where the paper quotes a 1e-5
suppression) and each variant takes the largest alpha whose measured 99th
percentile (10^4 random targets, FP64 direct summation on the device) meets the
bound: the first of a descending sqrt(2) grid that meets it, then three
bisections in log alpha towards the grid value above it.  `value` is the faster variant that meets it.

Extra keys: the same comparison on two more held-out boxes of the headline
size (seeds 2002 and 2003) and on the 128^3 box (seed 2), the as-stated
R_cut = 4.5 r_s, alpha = 0.005 line, the total TreePM force (that walk plus
the long-range PM force on the 256^3 mesh), the FMM at p = 3, theta = 0.5, the
batched forest of 64 boxes, and the FP64 oracle on the host cores.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle forces/s at 99th-pct rel. force err ≤1e-3 vs direct sum; learned vs plain"
PEAK_FP32_VECTOR = 157.3e12      # MI355X FP32 vector peak (assumes packed FP32 FMA), FLOP/s
PEAK_FP32_NONPACKED = 78.6e12    # 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz: what non-packed FMA can issue
ERR_BOUND = 1e-3
KEY_KINDS = {"morton": 0, "ph": 1}
ALPHAS = (0.004, 0.0028, 0.002, 0.0014, 0.001, 0.0007, 0.0005, 0.00035, 0.00025)
REFINE = 3  # bisections of the calibrated alpha between a passing grid value and the failing one above
HEADLINE_N = 256 ** 3
HEADLINE_SEED = 2001
SMALL_N = 128 ** 3
SMALL_SEED = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=HEADLINE_N, help="particles of the headline box")
    ap.add_argument("--seed", type=int, default=HEADLINE_SEED, help="generator seed of the headline box")
    ap.add_argument("--rcut", type=float, default=7.0, help="R_cut in units of r_s")
    ap.add_argument("--alpha", type=float, default=0.0, help="fix alpha for both variants instead of calibrating it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="CPU work the oracle baseline aims at")
    ap.add_argument("--no-as-stated", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the 128^3 comparison")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--eval-seeds", type=str, default="2002,2003",
                    help="further held-out seeds of the headline box for the same comparison ('' to skip)")
    ap.add_argument("--weights", type=str, default="", help="learned-seed weights (.npz); default by particle count")
    ap.add_argument("--no-fmm", action="store_true")
    ap.add_argument("--fmm-leaf", type=int, default=32,
                    help="leaf size of the second, tuned FMM line (the first keeps the configuration's leaf 16)")
    ap.add_argument("--no-forest", action="store_true")
    ap.add_argument("--no-pm", action="store_true", help="skip the total TreePM (walk + PM) line")
    ap.add_argument("--no-kdk", action="store_true", help="skip the hierarchical time-integration line")
    ap.add_argument("--no-ewald", action="store_true", help="skip the periodic tree + Ewald line")
    ap.add_argument("--no-orders", action="store_true", help="skip the expansion-order (p = 3, 4, 5) comparison")
    ap.add_argument("--err-sample", type=int, default=10000)
    ap.add_argument("--group", type=int, default=64)
    ap.add_argument("--leaf", type=int, default=32, help="leaf size B of the tree")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--keys", choices=("morton", "ph"), default="morton",
                    help="curve order of the particles: Morton or Peano-Hilbert (same nodes)")
    ap.add_argument("--sr-table", type=int, default=0,
                    help="intervals of the short-range factor table of the walks (0: erfc/exp per interaction)")
    ap.add_argument("--profile-fmm", type=int, default=0, metavar="LEAF",
                    help="only run `steps` calls of the FMM (atomic-sum mode) on the clustered 128^3 box (seed 3) at "
                         "this leaf size, for counter runs of its kernels")
    ap.add_argument("--profile-walk", choices=("plain", "learned"), default=None,
                    help="only time `steps` steps of this variant at --alpha on the headline box (no reference "
                         "sums, no calibration), for counter runs of the walk")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


WALK_SOURCES = ("walk.hip", "ewald.h", "g4_device.h", "g4_internal.h")


def traffic_file(n):
    side = round(n ** (1 / 3))
    return os.path.join(ROOT, "profiles", f"walk_treepm_clustered{side}_traffic.txt")


def walk_source_sha():
    """Hash of the walk's sources with comments and blank lines removed (so that
    a comment edit does not orphan the committed counter summary)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_03567_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(line.rstrip() for line in src.splitlines() if line.strip()).encode())
    return h.hexdigest()


def walk_traffic(n, variant, alpha, leaf):
    """HBM bytes per launch of the relative walk from the committed counter
    summary, if it was taken on the current walk sources for this box size,
    variant, alpha and leaf size; None otherwise."""
    path = traffic_file(n)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha256") != walk_source_sha() or kv.get("variant") != variant or \
                abs(float(kv.get("alpha", "nan")) - alpha) > 1e-12 or kv.get("leaf_max") != str(leaf):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def treepm_scales(n):
    """Split scale and softening of the clustered-box workload at n particles
    (fixed relative to the mean spacing: r_s = 1.25/256, eps0 = 1/(40*128) at 128^3)."""
    scale = (128 ** 3 / n) ** (1.0 / 3.0)
    return 1.25 / 256 * scale, scale / (40 * 128)


class TreePMCase:
    """One clustered periodic box resident on the device, with the plain
    (geometric pre-walk) and learned (MLP) seeding of the relative walk."""

    def __init__(self, g, ctx, args, n, seed, weights=""):
        import torch
        import workloads
        self.g, self.ctx, self.args, self.n, self.seed = g, ctx, args, n, seed
        self.r_s, self.eps0 = treepm_scales(n)
        self.r_cut = args.rcut * self.r_s
        log(f"[bench] generating clustered box n={n} seed={seed}")
        ps = workloads.clustered_box(n, seed=seed)
        self.ps = ps
        dev = ctx.device
        self.pos = torch.from_numpy(ps.pos).to(dev)
        self.mass = torch.from_numpy(ps.mass.astype(np.float32)).to(dev)
        self.tp = g.tree_params(True, ps.box, leaf_max=args.leaf, key_kind=KEY_KINDS[args.keys])
        self.ws = torch.empty(g.g4_workspace_bytes(self.tp, n) + 256, dtype=torch.uint8, device=dev)
        self.outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
        self.out = (*self.outs, None, None, None)
        self.stream = torch.cuda.current_stream(dev)
        self.state = {}
        self.learned = None
        wdir = os.path.join(ROOT, "paper_2010_03567_amd", "weights")
        wfile = weights or os.path.join(wdir, f"seed_mlp_{n}_leaf{args.leaf}.npz")
        if not args.no_learned and os.path.exists(wfile):
            from paper_2010_03567_amd import train_seed
            wl, norm, meta = train_seed.load(wfile, dev)
            if int(meta.get("leaf", 8)) == args.leaf:
                self.learned = dict(w=wl, norm=norm, meta=meta, file=os.path.basename(wfile),
                                    aseed=torch.empty(n, dtype=torch.float32, device=dev),
                                    feat=torch.empty((n, 8), dtype=torch.float32, device=dev),
                                    fwp=g.walk_params(kernel=1, r_s=self.r_s, eps0=self.eps0))
            else:
                log(f"[bench] {os.path.basename(wfile)} was trained on leaf {meta.get('leaf')}, not {args.leaf}")
        self.ref = None
        self.tg = None

    def params(self, variant, alpha, r_cut=None, order=3):
        """Walk parameters (pre-walk, relative walk); `order` is the relative
        walk's expansion order p (the pre-walk stays at p = 3)."""
        g, a = self.g, self.args
        kw = dict(kernel=1, r_s=self.r_s, r_cut=self.r_cut if r_cut is None else r_cut, eps0=self.eps0,
                  group_size=a.group, sr_table=a.sr_table)
        if variant == "plain":
            return (g.walk_params(criterion=0, theta=0.7, **kw),
                    g.walk_params(criterion=1, alpha=alpha, seed_from_tree=1, order=order, **kw))
        return (None, g.walk_params(criterion=1, alpha=alpha, a_seed=self.learned["aseed"], order=order, **kw))

    def step(self, variant, wps, evs=None, want_stats=False):
        """One pass of the path; evs: 4 events (start, after moments, after seed, after walk)."""
        g, ctx = self.g, self.ctx
        if evs is not None:
            evs[0].record(self.stream)
        x, y, z = g.g4_quantize(ctx, self.pos, self.tp)
        p = g.particles(x, y, z, self.mass)
        tree = g.g4_build_tree(ctx, p, self.tp, ws=self.ws)
        g.g4_compute_multipoles(ctx, tree, 3)
        if wps[1].order >= 4:
            import torch
            if self.state.get("m4") is None:
                self.state["m4"] = torch.empty(g.g4_moments4_bytes(tree) + 256, dtype=torch.uint8, device=ctx.device)
            g.g4_compute_moments4(ctx, tree, ws=self.state["m4"])
        if evs is not None:
            evs[1].record(self.stream)
        seed_stats = None
        if variant == "plain":
            seed_stats = g.g4_treepm_shortrange(ctx, tree, wps[0], out=self.out, want_stats=want_stats)["stats"]
        else:
            L = self.learned
            feat = g.g4_mlp_features(ctx, tree, L["fwp"], L["norm"], out=L["feat"])
            g.g4_mlp_forward(ctx, L["w"], feat, shift=0.0, mode=1, out=L["aseed"])
        if evs is not None:
            evs[2].record(self.stream)
        st = g.g4_treepm_shortrange(ctx, tree, wps[1], out=self.out, want_stats=want_stats)["stats"]
        if evs is not None:
            evs[3].record(self.stream)
        self.state["tree"], self.state["p"] = tree, p
        return seed_stats, st

    def reference(self):
        """FP64 direct summation (untruncated short-range q = 0 sum) on a random sample of targets."""
        import torch
        import workloads
        if self.ref is None:
            g = self.g
            self.step("plain", self.params("plain", 0.001))
            tg = workloads.sample_indices(self.n, self.args.err_sample, seed=99)
            self.tg = torch.from_numpy(tg).to(self.ctx.device)
            wpd = g.walk_params(kernel=1, r_s=self.r_s, r_cut=1e30, eps0=self.eps0)
            r = g.g4_direct_force(self.ctx, self.state["p"], self.tp, wpd, targets=self.tg, want_pot=False)
            self.ref = np.stack([r["ax"].cpu().numpy(), r["ay"].cpu().numpy(), r["az"].cpu().numpy()], 1)
        return self.ref

    def errors(self, variant, wps):
        import torch
        import workloads
        ref = self.reference()
        self.step(variant, wps)
        a = torch.stack(self.outs, 1)[self.tg].cpu().numpy()
        return workloads.percentiles(workloads.relative_errors(a, ref))

    def calibrate(self, variant, fixed=0.0, order=3):
        """The largest alpha whose p99 error meets the bound: the first grid value
        (descending by sqrt 2) that meets it, refined by REFINE bisections in
        log alpha towards the grid value above it, which failed."""
        cal, chosen = {}, None
        for i, a in enumerate((fixed,) if fixed > 0 else ALPHAS):
            cal[a] = self.errors(variant, self.params(variant, a, order=order))
            log(f"[bench] n={self.n} {variant} p={order} alpha={a}: {cal[a]}")
            if cal[a]["p99"] <= ERR_BOUND or fixed > 0:
                chosen = a
                if fixed <= 0 and i > 0:
                    lo, hi = a, ALPHAS[i - 1]
                    for _ in range(REFINE):
                        mid = float(f"{math.sqrt(lo * hi):.3g}")
                        if not lo < mid < hi:
                            break
                        cal[mid] = self.errors(variant, self.params(variant, mid, order=order))
                        log(f"[bench] n={self.n} {variant} p={order} alpha={mid}: {cal[mid]}")
                        if cal[mid]["p99"] <= ERR_BOUND:
                            lo = mid
                        else:
                            hi = mid
                    chosen = lo
                break
        return chosen, cal

    def timed(self, variant, wps, steps, warmup):
        """Wall time per step over exactly `steps` steps (synchronised on both
        sides) and the per-step event times of the phases."""
        import torch
        for _ in range(warmup):
            self.step(variant, wps)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(variant, wps, evs[k])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                        e[0].elapsed_time(e[3])] for e in evs])
        return ms, {"build_moments_ms": float(np.median(ph[:, 0])), "seed_ms": float(np.median(ph[:, 1])),
                    "walk_ms": float(np.median(ph[:, 2])), "walk_ms_mean": float(np.mean(ph[:, 2])),
                    "step_ms_median_events": float(np.median(ph[:, 3]))}

    def variant(self, variant, steps, warmup, fixed=0.0):
        alpha, cal = self.calibrate(variant, fixed)
        if alpha is None:
            return {"error": "no alpha in the grid met the error bound",
                    "alpha_calibration": {str(k): v["p99"] for k, v in cal.items()}}
        wps = self.params(variant, alpha)
        ms, ph = self.timed(variant, wps, steps, warmup)
        sst, st = self.step(variant, wps, want_stats=True)
        n = self.n
        res = {"alpha": alpha, "ms_per_step": ms, "forces_per_s": n / (ms * 1e-3), "phases": ph,
               "errors_vs_direct": cal[alpha], "alpha_calibration": {str(k): v["p99"] for k, v in cal.items()},
               "per_particle": {"p2p": st["n_p2p"] / n, "p2m": st["n_p2m"] / n, "visit": st["n_visit"] / n},
               "stats": st}
        if sst is not None:
            res["per_particle"].update(prewalk_p2p=sst["n_p2p"] / n, prewalk_p2m=sst["n_p2m"] / n,
                                       prewalk_visit=sst["n_visit"] / n)
        log(f"[bench] n={n} {variant}: {ms:.3f} ms/step at alpha {alpha} (seed {ph['seed_ms']:.3f} ms, walk "
            f"{ph['walk_ms']:.3f} ms), errors {cal[alpha]}")
        return res

    def compare(self, steps, warmup, fixed=0.0):
        out = {"workload": f"clustered box {round(self.n ** (1 / 3))}^3 (seed {self.seed}), R_cut {self.args.rcut} r_s, "
                           f"leaf {self.args.leaf}", "n": self.n, "seed": self.seed}
        out["plain"] = self.variant("plain", steps, warmup, fixed)
        if self.learned is not None:
            out["learned"] = self.variant("learned", steps, warmup, fixed)
            out["learned"]["weights"] = self.learned["file"]
            meta = self.learned["meta"]
            out["learned"]["trained_on"] = {k: meta.get(k) for k in ("n", "leaf", "seeds", "rcut", "alpha", "steps",
                                                                      "tau")}
            out["learned"]["train_residual_rms_dex"] = meta.get("residual_rms")
        if "ms_per_step" in out["plain"] and "ms_per_step" in out.get("learned", {}):
            out["speedup_learned_vs_plain"] = out["plain"]["ms_per_step"] / out["learned"]["ms_per_step"]
            # what skipping the pre-walk entirely could give: the plain step without its seed phase
            p = out["plain"]
            out["learned_ceiling_speedup"] = p["ms_per_step"] / (p["ms_per_step"] - p["phases"]["seed_ms"])
        return out

    def free(self):
        import torch
        self.state.clear()
        del self.ws, self.outs, self.out, self.pos, self.mass
        if self.learned is not None:
            self.learned.clear()
        torch.cuda.empty_cache()


def walk_roofline(flops, st, walk_ms, n, variant, alpha, leaf):
    """Roofline entry of the relative walk: algorithmic FLOPs at the
    per-interaction units of the measurement plan (particle-particle and
    particle-node interactions only) over the mean HIP-event duration."""
    alg = flops.walk_flops_algorithmic("treepm", st["n_p2m"], st["n_p2p"])
    visit = flops.VISIT_BOOKKEEPING[("treepm", "relative")] * float(st["n_visit"])
    achieved = alg / (walk_ms * 1e-3)
    return {"bound": "alu", "kernel": "k_walk<1,1,false,true> (relative TreePM walk, p = 3)",
            "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR, "traffic": walk_traffic(n, variant, alpha, leaf),
            "frac_of_nonpacked_issue_peak": achieved / PEAK_FP32_NONPACKED,
            "avg_ms": walk_ms, "flop_per_launch": alg,
            "flop_units": {"p2p": flops.P2P_ALG["treepm"], "p2m": flops.P2M_ALG["treepm"]},
            "visit_flop_not_counted": visit, "variant": variant, "alpha": alpha}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2010_03567_amd import flops
    import paper_2010_03567_amd.g4hip as g

    ctx = g.Context()
    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb * 2 ** 18, dtype=torch.float32, device=ctx.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.profile_fmm:
        print(json.dumps(profile_fmm(g, ctx, args.profile_fmm, args.steps, args.warmup)))
        return
    head = TreePMCase(g, ctx, args, args.n, args.seed, args.weights)
    if args.profile_walk:
        if args.alpha <= 0:
            raise SystemExit("--profile-walk needs --alpha")
        if args.profile_walk == "learned" and head.learned is None:
            raise SystemExit("no learned-seed weights for this particle count")
        ms, ph = head.timed(args.profile_walk, head.params(args.profile_walk, args.alpha), args.steps, args.warmup)
        print(json.dumps({"profile_walk": args.profile_walk, "n": args.n, "alpha": args.alpha, "steps": args.steps,
                          "ms_per_step": ms, "walk_ms": ph["walk_ms_mean"], "walk_source_sha256": walk_source_sha()}))
        return

    cmp = head.compare(args.steps, args.warmup, args.alpha)
    n = args.n
    ok = {k: cmp[k] for k in ("plain", "learned") if "ms_per_step" in cmp.get(k, {})}
    best = min(ok, key=lambda k: ok[k]["ms_per_step"])
    chosen = ok[best]
    st = chosen.pop("stats")
    for k in ok:
        ok[k].pop("stats", None)
    roof = walk_roofline(flops, st, chosen["phases"]["walk_ms_mean"], n, best, chosen["alpha"], args.leaf)
    # visit passes carry the pairs the targets decide one by one; pairs decided for a whole group
    # (used by every target, or dropped by every target) take no visit slot
    util = {"pop": (st["n_visit"] - st["n_group_use"]) / max(1, 64 * st["w_pop"]),
            "p2m": st["n_p2m"] / max(1, 64 * st["w_p2m"]), "p2p": st["n_p2p"] / max(1, 64 * st["w_p2p"])}
    side = round(n ** (1 / 3))
    result = {
        "metric": METRIC,
        "value": chosen["forces_per_s"],
        "unit": "forces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chosen["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"learned_vs_plain_treepm_clustered_box_{side}^3", "n": n, "seed": args.seed,
                   "box": 1.0, "r_s": head.r_s, "r_cut": head.r_cut, "R_cut": args.rcut, "eps0": head.eps0,
                   "leaf_max": args.leaf, "order": 3, "alpha": chosen["alpha"], "theta_seed": 0.7,
                   "group_size": args.group, "sr_table": args.sr_table, "keys": args.keys,
                   "variant": "learned (MLP |a| seed + relative walk)" if best == "learned"
                   else "plain (geometric pre-walk + relative walk)"},
        "comparison": cmp,
        "roofline": roof,
        "walk_counters": {"lane_utilisation": util,
                          "passes": {k: st[k] for k in ("w_pop", "w_p2m", "w_p2p", "w_entry", "w_leaf", "w_chunk",
                                                        "max_stack")},
                          "group_decided_per_particle": {"use": st["n_group_use"] / n,
                                                         "drop": st["n_group_drop"] / n}},
    }
    cpu_input = (head.ps, head.r_s, head.r_cut, head.eps0, chosen["alpha"])
    head.free()
    del head
    if args.eval_seeds:
        result["held_out_seeds"] = held_out_seeds(args, g, ctx)
    if not args.no_small and args.n != SMALL_N:
        small = TreePMCase(g, ctx, args, SMALL_N, SMALL_SEED)
        sc = small.compare(max(5, args.steps), 2, args.alpha)
        for k in ("plain", "learned"):
            if k in sc:
                sc[k].pop("stats", None)
        result["treepm_128^3"] = sc
        if not args.no_as_stated:
            wps45 = small.params("plain", 0.005, r_cut=4.5 * small.r_s)
            e45 = small.errors("plain", wps45)
            ms45, ph45 = small.timed("plain", wps45, 5, 1)
            result["as_stated_rcut4.5_alpha0.005_128^3"] = {"forces_per_s": SMALL_N / (ms45 * 1e-3),
                                                          "ms_per_step": ms45, "phases": ph45,
                                                          "errors_vs_direct": e45}
            log(f"[bench] as stated (128^3, R_cut 4.5, alpha 0.005): {ms45:.3f} ms/step, errors {e45}")
        if not args.no_pm:
            result["treepm_total_128^3"] = bench_total_treepm(args, g, ctx, small)
        if not args.no_orders:
            result["orders_128^3"] = bench_orders(args, small)
        small.free()
        del small
    if not args.no_fmm:
        result["fmm"] = bench_fmm(args, g, ctx, flops)
    if not args.no_kdk:
        result["hierarchical_step"] = bench_kdk(args, g, ctx)
    if not args.no_ewald:
        result["periodic_ewald"] = bench_ewald(args, g, ctx, flops)
    if not args.no_forest:
        result["forest"] = bench_forest(args, g, ctx)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(*cpu_input, args)
    print(json.dumps(result), flush=True)


def held_out_seeds(args, g, ctx):
    """The headline comparison (each variant at its own calibrated alpha) on
    further boxes of the same size drawn with other held-out seeds: the
    network, the loss and the leaf size were chosen on the headline box."""
    out = {}
    for seed in (int(x) for x in args.eval_seeds.split(",")):
        case = TreePMCase(g, ctx, args, args.n, seed, args.weights)
        c = case.compare(5, 2, args.alpha)
        case.free()
        del case
        row = {}
        for k in ("plain", "learned"):
            v = c.get(k, {})
            if "ms_per_step" in v:
                row[k] = {"alpha": v["alpha"], "ms_per_step": v["ms_per_step"], "errors_vs_direct": v["errors_vs_direct"],
                          "per_particle": v["per_particle"], "seed_ms": v["phases"]["seed_ms"],
                          "walk_ms": v["phases"]["walk_ms"]}
            elif v:
                row[k] = {"error": v.get("error")}
        for k in ("speedup_learned_vs_plain", "learned_ceiling_speedup"):
            if k in c:
                row[k] = c[k]
        out[str(seed)] = row
    return out


def bench_orders(args, case):
    """The relative TreePM walk at expansion orders p = 3, 4, 5 on the 128^3
    box (geometric pre-walk seeds, the pre-walk at p = 3), each at the largest
    alpha of the grid whose p99 error against the FP64 direct sum is <= 1e-3:
    a higher order costs more per interaction and allows a larger alpha."""
    out = {}
    for order in (3, 4, 5):
        alpha, cal = case.calibrate("plain", order=order)
        if alpha is None:
            out[f"p{order}"] = {"error": "no alpha in the grid met the error bound"}
            continue
        wps = case.params("plain", alpha, order=order)
        ms, ph = case.timed("plain", wps, max(3, args.steps // 2), 1)
        _, st = case.step("plain", wps, want_stats=True)
        n = case.n
        out[f"p{order}"] = {"alpha": alpha, "ms_per_step": ms, "walk_ms": ph["walk_ms"],
                            "errors_vs_direct": cal[alpha],
                            "per_particle": {"p2p": st["n_p2p"] / n, "p2m": st["n_p2m"] / n}}
        log(f"[bench] 128^3 plain p={order}: {ms:.3f} ms/step at alpha {alpha} (walk {ph['walk_ms']:.3f} ms), "
            f"p2m {st['n_p2m'] / n:.0f}, p2p {st['n_p2p'] / n:.0f} per particle")
    return out


def bench_total_treepm(args, g, ctx, case):
    """Total TreePM force on the 128^3 box as the configuration states it:
    short-range walk at R_cut = 4.5 r_s (geometric pre-walk, relative
    criterion at alpha = 0.005) plus the long-range PM force on the 256^3 mesh
    (r_s = 1.25 L/256).  Errors of the total force against the untruncated
    short-range direct sum plus the PM force on a 512^3 mesh at the same
    split (A_smth = 2.5: its own long-range error is about four times
    smaller, see the PM oracle's convergence pin), on 10^4 random targets."""
    import torch
    import workloads
    n = case.n
    sr_ref = case.reference()
    wps = case.params("plain", 0.005, r_cut=4.5 * case.r_s)
    pp = g.pm_params(256, case.r_s)
    state = {"ws": None}

    def step(evs=None):
        case.step("plain", wps, evs[:4] if evs else None)
        o = g.g4_pm_longrange(ctx, case.state["tree"], pp, ws=state["ws"], accumulate=True, out=case.outs + [None])
        state["ws"] = o["ws"]
        if evs:
            evs[4].record(case.stream)

    step()
    torch.cuda.synchronize()
    steps = max(5, args.steps // 2)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    pm_ms = float(np.median([e[3].elapsed_time(e[4]) for e in evs]))
    walk_ms = float(np.median([e[2].elapsed_time(e[3]) for e in evs]))
    a = torch.stack(case.outs, 1)
    # long-range reference: PM at twice the resolution, same split
    fine = g.g4_pm_longrange(ctx, case.state["tree"], g.pm_params(512, case.r_s))
    lr_fine = torch.stack([fine["ax"], fine["ay"], fine["az"]], 1)[case.tg].cpu().numpy()
    del fine
    torch.cuda.empty_cache()
    tot = a[case.tg].cpu().numpy()
    err = workloads.percentiles(workloads.relative_errors(tot, sr_ref + lr_fine))
    log(f"[bench] total TreePM 128^3 (R_cut 4.5, alpha 0.005, PM 256^3): {ms:.3f} ms/step (PM {pm_ms:.3f} ms), "
        f"errors {err}")
    return {"workload": "total TreePM force, clustered 128^3 box (seed 2), R_cut 4.5 r_s, alpha 0.005, PM mesh 256^3",
            "forces_per_s": n / (ms * 1e-3), "ms_per_step": ms, "pm_ms": pm_ms, "walk_ms": walk_ms,
            "errors_vs_reference": err,
            "reference": "untruncated short-range FP64 direct sum + PM at mesh 512^3 (A_smth 2.5)"}


def bench_kdk(args, g, ctx):
    """Hierarchical time integration on the clustered 128^3 box (seed 2, cold
    start): FMM forces (p = 3, theta = 0.5, leaf 16, short-range kernel at
    R_cut = 4.5 r_s), step criterion sqrt(2 eta eps / |a|) with eta = 0.025,
    eps = eps0, and dt_max = 8 x the median criterion step, so the haloes
    split over several levels.  Reported: time per step of dt_max, the levels
    used, force evaluations (every particle that received a force), the
    force-evaluation rate, and the paper's cost comparison with one-sided
    nesting (K_onesided = N_0 + sum_k 2^(k-1) N_k)."""
    import torch
    import workloads
    n = SMALL_N
    r_s, eps0 = treepm_scales(n)
    ps = workloads.clustered_box(n, seed=2)
    dev = ctx.device
    tp = g.tree_params(True, 1.0, leaf_max=16)
    fp = g.fmm_params(kernel=1, theta=0.5, r_s=r_s, r_cut=4.5 * r_s, eps0=eps0)
    eta = 0.025
    kp = g.kdk_params(2, tp, eta, eps0, max_level=12, fp=fp)
    pos0 = torch.from_numpy(ps.pos).to(dev)
    mass = torch.from_numpy(ps.mass.astype(np.float32)).to(dev)
    pos, vel = pos0.clone(), torch.zeros_like(pos0)
    acc, st, ws = g.g4_kdk_step(ctx, kp, pos, vel, mass, 1e-12)  # forces of the whole box (tiny step)
    amag = torch.sqrt(acc[0] ** 2 + acc[1] ** 2 + acc[2] ** 2).cpu().numpy()
    dt = 8.0 * float(np.median(np.sqrt(2 * eta * eps0 / np.maximum(amag, 1e-30))))
    acc0 = tuple(a.clone() for a in acc)  # forces at the start (the tiny step moved nothing measurably)
    pos.copy_(pos0)
    vel.zero_()
    acc, _, ws = g.g4_kdk_step(ctx, kp, pos, vel, mass, dt, acc=tuple(a.clone() for a in acc0), ws=ws)  # warm-up
    pos.copy_(pos0)
    vel.zero_()
    acc = tuple(a.clone() for a in acc0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc, st, ws = g.g4_kdk_step(ctx, kp, pos, vel, mass, dt, acc=acc, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    lv = st["evals_per_level"]
    # N_k: particles on level k or deeper = the set sizes of the first sub-step of each level
    nk = [n] + [lv[k] // (3 * 2 ** (k - 1)) for k in range(1, st["deepest_level"] + 1)]
    onesided = n + sum(2 ** (k - 1) * nk[k] for k in range(1, len(nk)))
    log(f"[bench] hierarchical step (FMM, 128^3): {ms:.1f} ms, levels {st['deepest_level']}, "
        f"force evaluations {st['force_evals']}")
    return {"workload": "hierarchical KDK step, clustered 128^3 box (seed 2), FMM p=3 theta 0.5 leaf 16, R_cut 4.5 r_s",
            "dt_max": dt, "ms_per_step": ms, "deepest_level": st["deepest_level"],
            "force_evals": st["force_evals"], "force_calls": st["force_calls"],
            "force_evals_per_s": st["force_evals"] / (ms * 1e-3), "evals_per_level": lv[: st["deepest_level"] + 1],
            "cost_vs_onesided": st["force_evals"] / onesided if onesided else None,
            "note": "one step from rest; the forces at the start are given (as in a running integration)"}


def bench_ewald(args, g, ctx, flops):
    """Periodic gravity by the pure tree with the Ewald correction (kernel 2)
    on the clustered 128^3 box (seed 2): the correction table (ne = 32) built
    once per box size, then per step build, moments, geometric pre-walk
    (theta 0.7) and the relative walk (p = 3, alpha 0.002); errors against the
    exact Ewald direct sum (FP64, every pair summed by Ewald's method) on
    sampled targets."""
    import torch
    import workloads
    n = SMALL_N
    _, eps0 = treepm_scales(n)
    ps = workloads.clustered_box(n, seed=2)
    dev = ctx.device
    pos = torch.from_numpy(ps.pos).to(dev)
    mass = torch.from_numpy(ps.mass.astype(np.float32)).to(dev)
    tp = g.tree_params(True, 1.0, leaf_max=args.leaf)
    ws = torch.empty(g.g4_workspace_bytes(tp, n) + 256, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    table = g.EwaldTable(ctx, 1.0, 32)
    torch.cuda.synchronize()
    table_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] periodic tree + Ewald: table (ne 32) built in {table_ms:.1f} ms")
    alpha = 0.002
    wp = g.walk_params(kernel=2, criterion=1, alpha=alpha, theta_seed=0.7, eps0=eps0, group_size=args.group,
                       ewald=table)
    outs = tuple(torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)) + (None, None, None)
    state = {}

    def step(want_stats=False):
        x, y, z = g.g4_quantize(ctx, pos, tp)
        p = g.particles(x, y, z, mass)
        t = g.g4_build_tree(ctx, p, tp, ws=ws)
        g.g4_compute_multipoles(ctx, t, 3)
        o = g.g4_tree_force(ctx, t, wp, out=outs, want_stats=want_stats)
        state["p"], state["o"] = p, o
        if want_stats:
            state["stats"] = o["stats"]

    step(want_stats=True)
    log(f"[bench] periodic tree + Ewald: first step done")
    steps = max(2, args.steps // 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = state["stats"]
    log(f"[bench] periodic tree + Ewald: {ms:.2f} ms/step; exact Ewald direct sums on 256 targets")
    a = np.stack([outs[0].cpu().numpy(), outs[1].cpu().numpy(), outs[2].cpu().numpy()], 1)
    tg = workloads.sample_indices(n, 256, seed=97)
    r = g.g4_direct_force(ctx, state["p"], tp, g.walk_params(kernel=2, eps0=eps0),
                          targets=torch.from_numpy(tg).to(dev), want_pot=False)
    ref = np.stack([r["ax"].cpu().numpy(), r["ay"].cpu().numpy(), r["az"].cpu().numpy()], 1)
    err = workloads.percentiles(workloads.relative_errors(a[tg], ref))
    # the periodic FMM with the same table (theta 0.5, leaf 32, atomic-sum mode)
    tpf = g.tree_params(True, 1.0, leaf_max=32)
    wsf = torch.empty(g.g4_workspace_bytes(tpf, n) + 256, dtype=torch.uint8, device=dev)
    fp = g.fmm_params(kernel=2, theta=0.5, eps0=eps0, ewald=table)
    fst = {"factor": 1.0, "fws": None}

    def fstep():
        x, y, z = g.g4_quantize(ctx, pos, tpf)
        t = g.g4_build_tree(ctx, g.particles(x, y, z, mass), tpf, ws=wsf)
        g.g4_compute_multipoles(ctx, t, 3)
        o = g.g4_fmm_force(ctx, t, fp, list_factor=fst["factor"], ws=fst["fws"])
        fst["factor"], fst["fws"], fst["o"] = o["list_factor"], o["ws"], o

    fstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fstep()
    torch.cuda.synchronize()
    fmm_ms = (time.perf_counter() - t0) * 1e3 / steps
    o = fst["o"]
    af = np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)
    ferr = workloads.percentiles(workloads.relative_errors(af[tg], ref))
    log(f"[bench] periodic FMM + Ewald 128^3 (theta 0.5, leaf 32): {fmm_ms:.2f} ms/step, errors {ferr}")
    walk_ms, seed_ms = 1e3 * st["t_walk"], 1e3 * st["t_seed"]
    log(f"[bench] periodic tree + Ewald 128^3: {ms:.2f} ms/step (walk {walk_ms:.2f} ms, pre-walk "
        f"{seed_ms:.2f} ms; table {table_ms:.1f} ms once), errors {err}")
    return {"workload": "periodic_tree_ewald_clustered_box_128^3 (seed 2), p=3, relative alpha 0.002 "
                        "(pre-walk theta 0.7), leaf %d, Ewald table ne 32" % args.leaf,
            "forces_per_s": n / (ms * 1e-3), "ms_per_step": ms, "walk_ms": walk_ms, "seed_ms": seed_ms,
            "table_build_ms": table_ms,
            "interactions_per_particle": {"pp": st["n_p2p"] / n, "pn": st["n_p2m"] / n,
                                          "seed_pp": st["n_seed_p2p"] / n, "seed_pn": st["n_seed_p2m"] / n},
            "errors_vs_ewald_direct": err, "error_sample": len(tg),
            "fmm": {"workload": "periodic FMM + Ewald, same box, p=3, theta 0.5, leaf 32, atomic-sum mode",
                    "ms_per_step": fmm_ms, "forces_per_s": n / (fmm_ms * 1e-3), "errors_vs_ewald_direct": ferr}}


def profile_fmm(g, ctx, leaf, steps, warmup):
    """FMM calls alone (tree built once) on the clustered 128^3 box of the FMM
    line, for kernel traces and counters; HIP-event time per call."""
    import torch
    import workloads
    n = SMALL_N
    r_s, eps0 = treepm_scales(n)
    ps = workloads.clustered_box(n, seed=3)
    pos = torch.from_numpy(ps.pos).to(ctx.device)
    mass = torch.from_numpy(ps.mass.astype(np.float32)).to(ctx.device)
    tp = g.tree_params(True, 1.0, leaf_max=leaf)
    x, y, z = g.g4_quantize(ctx, pos, tp)
    t = g.g4_build_tree(ctx, g.particles(x, y, z, mass), tp)
    g.g4_compute_multipoles(ctx, t, 3)
    fp = g.fmm_params(kernel=1, theta=0.5, r_s=r_s, r_cut=4.5 * r_s, eps0=eps0)
    st = {"factor": 1.0, "fws": None}
    evs = []
    for k in range(warmup + steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        o = g.g4_fmm_force(ctx, t, fp, list_factor=st["factor"], ws=st["fws"], want_stats=(k == 0))
        ev[1].record()
        st["factor"], st["fws"] = o["list_factor"], o["ws"]
        if k == 0:
            s0 = o["stats"]
        if k >= warmup:
            evs.append(ev)
    torch.cuda.synchronize()
    return {"profile_fmm": leaf, "n": n, "steps": steps, "fmm_ms": float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
            "per_particle": {"pp": s0["n_pp"] / n, "pn": s0["n_pn"] / n, "nn": s0["n_nn"] / n}}


def bench_fmm(args, g, ctx, flops):
    """Symmetric FMM (p = 3, theta = 0.5) on the clustered 128^3 box drawn with
    its own seed (3), short-range kernel at the same split, R_cut = 4.5 r_s:
    leaf 16 as the configuration states (atomic-sum mode timed per step, the
    sorted-list, bitwise reproducible mode timed alongside), and the
    atomic-sum mode again at the leaf size that measured fastest (--fmm-leaf)."""
    import torch
    import workloads
    n = SMALL_N
    r_s, eps0 = treepm_scales(n)
    ps = workloads.clustered_box(n, seed=3)
    dev = ctx.device
    pos = torch.from_numpy(ps.pos).to(dev)
    m32 = ps.mass.astype(np.float32)
    mass = torch.from_numpy(m32).to(dev)
    tg = workloads.sample_indices(n, args.err_sample, seed=98)
    ref = {}

    def case(leaf, with_sorted):
        tp = g.tree_params(True, 1.0, leaf_max=leaf)
        ws = torch.empty(g.g4_workspace_bytes(tp, n) + 256, dtype=torch.uint8, device=dev)

        def run(det, steps):
            fp = g.fmm_params(kernel=1, theta=0.5, r_s=r_s, r_cut=4.5 * r_s, eps0=eps0, deterministic=det)
            state = {"factor": 1.0, "fws": None}

            def step(ev=None):
                x, y, z = g.g4_quantize(ctx, pos, tp)
                p = g.particles(x, y, z, mass)
                t = g.g4_build_tree(ctx, p, tp, ws=ws)
                g.g4_compute_multipoles(ctx, t, 3)
                if ev is not None:
                    ev[0].record()
                o = g.g4_fmm_force(ctx, t, fp, list_factor=state["factor"], ws=state["fws"], want_stats=ev is None)
                if ev is not None:
                    ev[1].record()
                state["factor"], state["fws"], state["out"], state["p"] = o["list_factor"], o["ws"], o, p
                if o["stats"] is not None:
                    state["stats"] = o["stats"]

            step()
            evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                step(evs[k])
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            return ms, float(np.mean([e[0].elapsed_time(e[1]) for e in evs])), state

        ms, fmm_ms, state = run(0, max(3, args.steps // 2))
        o = state["out"]
        a = np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)
        net = float(np.abs((m32[:, None].astype(np.float64) * a).sum(0)).max() / (m32[:, None] * np.abs(a)).sum())
        if "a" not in ref:
            r = g.g4_direct_force(ctx, state["p"], tp, g.walk_params(kernel=1, r_s=r_s, eps0=eps0),
                                  targets=torch.from_numpy(tg).to(dev), want_pot=False)
            ref["a"] = np.stack([r["ax"].cpu().numpy(), r["ay"].cpu().numpy(), r["az"].cpu().numpy()], 1)
        st = state["stats"]
        alg = flops.fmm_flops_algorithmic(st["n_pp"], st["n_pn"], st["n_nn"], st["n_nodes"], n)
        res = {"workload": f"fmm_clustered_box_128^3 (seed 3), p=3, theta=0.5, leaf {leaf}, R_cut 4.5 r_s",
               "forces_per_s": n / (ms * 1e-3), "ms_per_step": ms, "fmm_ms": fmm_ms,
               "interactions_per_particle": {"pp": st["n_pp"] / n, "pn": st["n_pn"] / n, "nn": st["n_nn"] / n},
               "net_force_over_sum_abs": net, "list_factor": state["factor"],
               "errors_vs_direct": workloads.percentiles(workloads.relative_errors(a[tg], ref["a"])),
               "roofline": {"bound": "alu", "kernel": "whole FMM call (all kernels)", "unit": "TFLOP/s",
                            "achieved": alg / (fmm_ms * 1e-3) / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                            "frac": alg / (fmm_ms * 1e-3) / PEAK_FP32_VECTOR, "flop_per_call": alg,
                            "flop_units": flops.FMM_ALG}}
        msg = f"[bench] fmm leaf {leaf}: {ms:.3f} ms/step (fmm {fmm_ms:.3f} ms"
        if with_sorted:
            ms_det, fmm_det_ms, _ = run(1, 2)
            res["deterministic_mode"] = {"ms_per_step": ms_det, "fmm_ms": fmm_det_ms}
            msg += f"; sorted-list mode {fmm_det_ms:.3f} ms"
        log(msg + f"), net force {net:.2e}")
        return res

    out = case(16, True)
    if args.fmm_leaf != 16:
        out["tuned_leaf"] = case(args.fmm_leaf, False)
    out["relative_criterion"] = fmm_relative(args, g, ctx, pos, mass, n, r_s, eps0, tg, ref["a"])
    return out


def fmm_relative(args, g, ctx, pos, mass, n, r_s, eps0, tg, ref):
    """The FMM with the relative node-node criterion at leaf 32 (seeds: |a| of
    a geometric FMM call on the same box), at alpha 0.004 and 0.002, errors on
    the same targets."""
    import torch
    import workloads
    dev = ctx.device
    tp = g.tree_params(True, 1.0, leaf_max=32)
    ws = torch.empty(g.g4_workspace_bytes(tp, n) + 256, dtype=torch.uint8, device=dev)
    base = dict(kernel=1, theta=0.5, r_s=r_s, r_cut=4.5 * r_s, eps0=eps0)
    st = {"factor": 1.0, "fws": None}

    def call(fp):
        x, y, z = g.g4_quantize(ctx, pos, tp)
        t = g.g4_build_tree(ctx, g.particles(x, y, z, mass), tp, ws=ws)
        g.g4_compute_multipoles(ctx, t, 3)
        o = g.g4_fmm_force(ctx, t, fp, list_factor=st["factor"], ws=st["fws"], want_stats=True)
        st["factor"], st["fws"] = o["list_factor"], o["ws"]
        return o

    o = call(g.fmm_params(**base))
    seed = torch.sqrt(o["ax"] ** 2 + o["ay"] ** 2 + o["az"] ** 2).float()
    res = {}
    for alpha in (0.004, 0.002):
        fp = g.fmm_params(criterion=1, alpha=alpha, a_seed=seed, **base)
        call(fp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = max(3, args.steps // 2)
        for _ in range(steps):
            o = call(fp)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        a = np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)
        err = workloads.percentiles(workloads.relative_errors(a[tg], ref))
        s = o["stats"]
        res[str(alpha)] = {"ms_per_step": ms, "errors_vs_direct": err,
                           "interactions_per_particle": {"pp": s["n_pp"] / n, "pn": s["n_pn"] / n, "nn": s["n_nn"] / n}}
        log(f"[bench] fmm relative (leaf 32) alpha {alpha}: {ms:.2f} ms/step, errors {err}")
    return res


def bench_forest(args, g, ctx):
    """Batched persistent walk over 64 independent clustered boxes (N log-uniform
    in [32768, 1048576], seeds 3000+b, concentration spread x3), leaf and group
    size from the autotuner's table when present; force errors against FP64
    direct summation on random targets spread over all boxes."""
    import workloads
    from paper_2010_03567_amd.autotune import ForestStep
    boxes = workloads.forest(64, seed=3000)
    r_s = 1.25 / 256
    tf = os.path.join(ROOT, "paper_2010_03567_amd", "weights", "autotune_forest.json")
    B, G, alpha, tuned = 8, 64, 0.001, False
    if os.path.exists(tf):
        with open(tf) as fh:
            t = json.load(fh)
        B, G, tuned = int(t["B"]), int(t["G"]), True
        alpha = float(t.get("alpha_chosen", t.get("alpha", alpha)))
    step = ForestStep(ctx, boxes, r_s, args.rcut * r_s, 1.0 / (40 * 128), alpha)
    ms, pre, walk = step.time(B, G, steps=max(3, args.steps // 2))
    err = step.errors(B, G, args.err_sample)
    log(f"[bench] forest: {step.n} particles in 64 boxes, {ms:.3f} ms/step (B={B}, G={G}), errors {err}")
    return {"workload": "forest of 64 clustered boxes", "n": step.n, "forces_per_s": step.n / (ms * 1e-3),
            "ms_per_step": ms, "prewalk_ms": pre, "walk_ms": walk, "leaf_max": B, "group_size": G,
            "autotuned": tuned, "R_cut": args.rcut, "alpha": alpha, "errors_vs_direct": err}


def cpu_baseline(ps, r_s, r_cut, eps0, alpha, args):
    """The FP64 oracle (built -O3 -march=native on this host) on all host
    cores: quantise + tree + moments over every particle, then pre-walk +
    relative walk for a random sample of targets sized to about
    --cpu-seconds of walking, scaled per particle to the whole box."""
    import platform
    import oracle
    import workloads
    oracle.select(native=True)
    threads = os.cpu_count() or 1
    try:
        model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")),
                     platform.processor())
    except OSError:
        model = platform.processor()
    n = ps.pos.shape[0]
    B = args.leaf
    t0 = time.perf_counter()
    st, X, Y, Z = oracle.quantize(ps.pos, True, ps.box)
    t = oracle.Tree(X, Y, Z, ps.mass.astype(np.float32).astype(np.float64), True, ps.box, B, nthreads=threads)
    t.compute_moments(nthreads=threads)
    t1 = time.perf_counter()
    kw = dict(kernel=1, r_s=r_s, r_cut=r_cut, eps0=eps0, nthreads=threads, want_pot=False)

    def walks(tg, nth):
        k = dict(kw, targets=tg, nthreads=nth)
        a0, _, _ = t.walk(criterion=0, theta=0.7, **k)
        seed = np.zeros(n)
        seed[tg] = np.linalg.norm(a0, axis=1)
        t.walk(criterion=1, alpha=alpha, aseed=seed, **k)

    # a small probe sizes the sample to the requested CPU time
    probe = workloads.sample_indices(n, 20 * threads, seed=4)
    tp0 = time.perf_counter()
    walks(probe, threads)
    per = (time.perf_counter() - tp0) / len(probe)
    k = int(min(n, max(1000, args.cpu_seconds / max(per, 1e-9))))
    tg = workloads.sample_indices(n, k, seed=5)
    t2 = time.perf_counter()
    walks(tg, threads)
    t3 = time.perf_counter()
    total = (t1 - t0) + (t3 - t2) * n / len(tg)
    log(f"[bench] oracle ({threads} threads, {model}): build+moments {t1 - t0:.2f} s, walks on {len(tg)} targets "
        f"{t3 - t2:.2f} s")
    # one thread, as the paper's single-core timings: the walks on a slice of the sample
    tg1 = tg[: max(1, len(tg) // threads)]
    t4 = time.perf_counter()
    walks(tg1, 1)
    t5 = time.perf_counter()
    return {"value": n / total, "unit": "forces/s", "cores": threads, "kind": "oracle", "cpu_model": model,
            "build": "gcc -O3 -march=native, pthreads",
            "sample": f"quantise+tree+moments over all {n} particles of the headline box ({t1 - t0:.1f} s) + "
                      f"pre-walk and relative walk (same R_cut, alpha {alpha}) for {len(tg)} random targets "
                      f"({t3 - t2:.1f} s), scaled to {n}",
            "single_thread_walk": {"forces_per_s_walk_only": len(tg1) / (t5 - t4), "cores": 1,
                                   "sample": f"pre-walk + relative walk for {len(tg1)} of the targets on one thread "
                                             f"({t5 - t4:.1f} s)"}}


if __name__ == "__main__":
    main()
