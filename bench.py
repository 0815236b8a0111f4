#!/usr/bin/env python3
"""Benchmark of the gravity hot path on one MI355X.

A step is one pass of the whole path over the clustered periodic 128^3 box:
integer mapping -> Morton keys + radix sort -> octree -> multipoles ->
geometric pre-walk (|a| seed, theta = 0.7) -> relative TreePM short-range walk
(alpha = 0.005) -> forces in the caller's order.  Inputs are resident in HBM
before the timed region.  Prints one JSON line.
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
PEAK_FP32_VECTOR = 157.3e12  # MI355X FP32 vector peak, FLOP/s
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128 ** 3)
    ap.add_argument("--alpha", type=float, default=0.005)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=20000)
    ap.add_argument("--err-sample", type=int, default=10000)
    ap.add_argument("--group", type=int, default=64)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads
    from paper_2010_03567_amd import flops
    import paper_2010_03567_amd.g4hip as g

    n = args.n
    scale = (128 ** 3 / n) ** (1.0 / 3.0)
    r_s = 1.25 / 256 * scale
    r_cut = 4.5 * r_s
    eps0 = scale / (40 * 128)
    B = 8
    log(f"[bench] generating clustered box n={n}")
    ps = workloads.clustered_box(n, seed=2)
    dev = torch.device("cuda", 0)
    ctx = g.Context()
    pos = torch.from_numpy(ps.pos).to(dev)
    mass = torch.from_numpy(ps.mass.astype(np.float32)).to(dev)
    tp = g.tree_params(True, ps.box, leaf_max=B)
    ws = torch.empty(g.g4_workspace_bytes(tp, n) + 256, dtype=torch.uint8, device=dev)
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
    out = (*outs, None, None, None)
    wp_seed = g.walk_params(kernel=1, criterion=0, theta=0.7, r_s=r_s, r_cut=r_cut, eps0=eps0, group_size=args.group)
    wp_rel = g.walk_params(kernel=1, criterion=1, alpha=args.alpha, r_s=r_s, r_cut=r_cut, eps0=eps0,
                           seed_from_tree=1, group_size=args.group)
    stream = torch.cuda.current_stream(dev)
    state = {}

    def step(evs=None):
        x, y, z = g.g4_quantize(ctx, pos, tp)
        p = g.particles(x, y, z, mass)
        tree = g.g4_build_tree(ctx, p, tp, ws=ws)
        g.g4_compute_multipoles(ctx, tree, 3)
        if evs is not None:
            evs[0].record(stream)
        g.g4_treepm_shortrange(ctx, tree, wp_seed, out=out)
        if evs is not None:
            evs[1].record(stream)
        g.g4_treepm_shortrange(ctx, tree, wp_rel, out=out)
        if evs is not None:
            evs[2].record(stream)
        state["tree"], state["p"] = tree, p
        return tree

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    # HIP events on the library's stream (torch's current stream), one triple per step
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    seed_avg_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    walk_avg_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    log(f"[bench] {ms_per_step:.3f} ms/step; walk {walk_avg_ms:.3f} ms, pre-walk {seed_avg_ms:.3f} ms")

    # interaction counts of one step (deterministic) for the algorithmic FLOPs
    tree, p = state["tree"], state["p"]
    st_seed = g.g4_treepm_shortrange(ctx, tree, wp_seed, out=out, want_stats=True)["stats"]
    st = g.g4_treepm_shortrange(ctx, tree, wp_rel, out=out, want_stats=True)["stats"]
    walk_flop = flops.walk_flops("treepm", "relative", st["n_visit"], st["n_p2m"], st["n_p2p"])
    seed_flop = flops.walk_flops("treepm", "geometric", st_seed["n_visit"], st_seed["n_p2m"], st_seed["n_p2p"])
    achieved = walk_flop / (walk_avg_ms * 1e-3)

    # force errors of the timed configuration against direct summation (FP64, on the GPU)
    ax = torch.stack(outs, 1).cpu().numpy()
    tg_np = workloads.sample_indices(n, args.err_sample, seed=99)
    tg = torch.from_numpy(tg_np).to(dev)
    wpd = g.walk_params(kernel=1, r_s=r_s, r_cut=r_cut, eps0=eps0)
    ref_u = g.g4_direct_force(ctx, p, tp, wpd, targets=tg, want_pot=False)
    ref_t = g.g4_direct_force(ctx, p, tp, wpd, targets=tg, truncate=True, want_pot=False)
    st3 = lambda o: np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)
    e_u = workloads.relative_errors(ax[tg_np], st3(ref_u))
    e_t = workloads.relative_errors(ax[tg_np], st3(ref_t))
    errors = {"vs_direct_untruncated": workloads.percentiles(e_u), "vs_direct_truncated_rcut": workloads.percentiles(e_t),
              "sample": int(len(tg_np))}
    log(f"[bench] errors {errors}")

    result = {
        "metric": METRIC,
        "value": n / (ms_per_step * 1e-3),
        "unit": "forces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "treepm_shortrange_clustered_box_128^3", "n": n, "box": 1.0, "r_s": r_s,
                   "r_cut": r_cut, "eps0": eps0, "leaf_max": B, "order": 3, "alpha": args.alpha, "theta_seed": 0.7,
                   "group_size": args.group, "variant": "plain (geometric pre-walk + relative walk)"},
        "roofline": {"bound": "alu", "kernel": "k_walk<1,1,false> (relative TreePM walk)", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
                     "traffic": None, "avg_ms": walk_avg_ms, "flop_per_launch": walk_flop},
        "breakdown_ms": {"prewalk": seed_avg_ms, "walk": walk_avg_ms},
        "interactions": {"walk": st, "prewalk": st_seed, "per_particle_p2p": st["n_p2p"] / n,
                         "per_particle_p2m": st["n_p2m"] / n},
        "errors": errors,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(ps, n, B, r_s, r_cut, eps0, args)
    print(json.dumps(result), flush=True)


def cpu_baseline(ps, n, B, r_s, r_cut, eps0, args):
    """The FP64 oracle timed on the host cores: tree build + moments over all n
    particles, then pre-walk + relative walk on a random sample of targets,
    scaled per particle to n."""
    import oracle
    import workloads
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    st, X, Y, Z = oracle.quantize(ps.pos, True, ps.box)
    t = oracle.Tree(X, Y, Z, ps.mass.astype(np.float32).astype(np.float64), True, ps.box, B)
    t.compute_moments()
    t1 = time.perf_counter()
    tg = workloads.sample_indices(n, args.cpu_sample, seed=5)
    kw = dict(kernel=1, r_s=r_s, r_cut=r_cut, eps0=eps0, nthreads=threads, targets=tg, want_pot=False)
    a0, _, _ = t.walk(criterion=0, theta=0.7, **kw)
    seed = np.zeros(n)
    seed[tg] = np.linalg.norm(a0, axis=1)
    t.walk(criterion=1, alpha=args.alpha, aseed=seed, **kw)
    t2 = time.perf_counter()
    total = (t1 - t0) + (t2 - t1) * n / len(tg)
    log(f"[bench] oracle: build+moments {t1 - t0:.2f} s, walks on {len(tg)} targets {t2 - t1:.2f} s")
    return {"value": n / total, "unit": "forces/s", "cores": threads, "kind": "oracle",
            "sample": f"quantise+tree+moments over all {n} particles ({t1 - t0:.1f} s) + pre-walk and relative "
                      f"walk for {len(tg)} random targets ({t2 - t1:.1f} s) scaled to {n}"}


if __name__ == "__main__":
    main()
