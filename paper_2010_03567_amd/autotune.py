"""Autotuner for the batched persistent walk: picks the leaf size B of the
tree and the particle-group size G of the walk's wavefront groups by timing
the whole step (forest build, multipoles, geometric pre-walk, relative walk)
on the workload itself, at equal accuracy: the leaf size changes the tree and
so the error at a given alpha, so for every B the largest alpha of a sqrt(2)
grid whose 99th-percentile force error against FP64 direct summation is at
most 1e-3 is found first, and the group sizes are timed at that alpha (the
group size changes the work packing, not the decisions).  G is capped at the
64 lanes of a wavefront.  The table and the choice are written as JSON.

    python -m paper_2010_03567_amd.autotune --out paper_2010_03567_amd/weights/autotune_forest.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
import paper_2010_03567_amd.g4hip as g  # noqa: E402

LEAVES = (4, 8, 16, 24, 32)
GROUPS = (16, 32, 48, 64)
ALPHAS = (0.004, 0.0028, 0.002, 0.0014, 0.001, 0.0007, 0.0005, 0.00035)
ERR_BOUND = 1e-3


class ForestStep:
    """One pass of the batched path over a fixed forest (inputs resident on the device)."""

    def __init__(self, ctx, boxes, r_s, r_cut, eps0, alpha, theta_seed=0.7):
        self.ctx = ctx
        dev = ctx.device
        self.n = int(sum(b.pos.shape[0] for b in boxes))
        self.off = np.concatenate([[0], np.cumsum([b.pos.shape[0] for b in boxes])]).astype(np.int64)
        self.pos = torch.from_numpy(np.concatenate([b.pos for b in boxes])).to(dev)
        self.mass = torch.from_numpy(np.concatenate([b.mass for b in boxes]).astype(np.float32)).to(dev)
        self.kw = dict(r_s=r_s, r_cut=r_cut, eps0=eps0)
        self.alpha, self.theta_seed = alpha, theta_seed
        self.outs = [torch.empty(self.n, dtype=torch.float64, device=dev) for _ in range(3)]
        self.ws = {}
        self.ref = None

    def reference(self, nsample):
        """FP64 direct summation (untruncated short-range sum within each box) on
        random targets spread over the boxes in proportion to their size."""
        if self.ref is None:
            ctx, dev = self.ctx, self.ctx.device
            tp = g.tree_params(True, 1.0, leaf_max=8)
            x, y, z = g.g4_quantize(ctx, self.pos, tp)
            wpd = g.walk_params(kernel=1, r_s=self.kw["r_s"], r_cut=1e30, eps0=self.kw["eps0"])
            tg_all, ref = [], []
            for b in range(len(self.off) - 1):
                lo, hi = int(self.off[b]), int(self.off[b + 1])
                k = max(8, int(round(nsample * (hi - lo) / self.n)))
                tg = workloads.sample_indices(hi - lo, k, seed=500 + b)
                p = g.particles(x[lo:hi], y[lo:hi], z[lo:hi], self.mass[lo:hi])
                r = g.g4_direct_force(ctx, p, tp, wpd, targets=torch.from_numpy(tg).to(dev), want_pot=False)
                ref.append(torch.stack([r["ax"], r["ay"], r["az"]], 1).cpu().numpy())
                tg_all.append(tg + lo)
            self.tg = torch.from_numpy(np.concatenate(tg_all)).to(dev)
            self.ref = np.concatenate(ref)
        return self.ref

    def errors(self, B, G, nsample=10000, alpha=None):
        """Percentiles of the relative force error of one step against the reference."""
        ref = self.reference(nsample)
        if alpha is not None:
            self.alpha = alpha
        self.run(B, G)
        a = torch.stack(self.outs, 1)[self.tg].cpu().numpy()
        return workloads.percentiles(workloads.relative_errors(a, ref))

    def run(self, B, G, evs=None):
        ctx = self.ctx
        tp = g.tree_params(True, 1.0, leaf_max=B)
        if B not in self.ws:
            self.ws[B] = torch.empty(g.g4_forest_workspace_bytes(tp, len(self.off) - 1, self.n) + 256,
                                     dtype=torch.uint8, device=ctx.device)
        x, y, z = g.g4_quantize(ctx, self.pos, tp)
        p = g.particles(x, y, z, self.mass)
        f = g.g4_build_forest(ctx, self.off, p, tp, ws=self.ws[B])
        g.g4_compute_multipoles(ctx, f, 3)
        out = (*self.outs, None, None, None)
        if evs is not None:
            evs[0].record()
        g.g4_treepm_shortrange(ctx, f, g.walk_params(kernel=1, criterion=0, theta=self.theta_seed, group_size=G,
                                                     **self.kw), out=out)
        if evs is not None:
            evs[1].record()
        g.g4_treepm_shortrange(ctx, f, g.walk_params(kernel=1, criterion=1, alpha=self.alpha, seed_from_tree=1,
                                                     group_size=G, **self.kw), out=out)
        if evs is not None:
            evs[2].record()
        self.forest, self.p = f, p
        return f

    def time(self, B, G, steps=3, warmup=1):
        for _ in range(warmup):
            self.run(B, G)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            self.run(B, G, evs[k])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        return ms, float(np.mean([e[0].elapsed_time(e[1]) for e in evs])), float(
            np.mean([e[1].elapsed_time(e[2]) for e in evs]))


def tune(step: ForestStep, leaves=LEAVES, groups=GROUPS, steps=3, log=print, nsample=10000):
    table = []
    for B in leaves:
        alpha, err = None, None
        for a in ALPHAS:
            e = step.errors(B, 64, nsample, alpha=a)
            log(f"[autotune] B={B} alpha={a}: {e}")
            if e["p99"] <= ERR_BOUND:
                alpha, err = a, e
                break
        if alpha is None:
            continue
        step.alpha = alpha
        for G in groups:
            ms, pre, walk = step.time(B, G, steps=steps)
            table.append(dict(B=B, G=G, alpha=alpha, errors=err, ms_per_step=ms, prewalk_ms=pre, walk_ms=walk))
            log(f"[autotune] B={B} G={G} alpha={alpha}: {ms:.2f} ms/step (pre-walk {pre:.2f}, walk {walk:.2f})")
    best = min(table, key=lambda r: r["ms_per_step"])
    return dict(B=best["B"], G=best["G"], alpha_chosen=best["alpha"], errors=best["errors"], table=table)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nbox", type=int, default=64)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--rcut", type=float, default=7.0)
    ap.add_argument("--alpha", type=float, default=0.001)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--out", type=str, required=True)
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    boxes = workloads.forest(a.nbox, seed=a.seed)
    log(f"[autotune] forest of {len(boxes)} boxes, {sum(b.pos.shape[0] for b in boxes)} particles")
    r_s = 1.25 / 256
    step = ForestStep(g.Context(), boxes, r_s, a.rcut * r_s, 1.0 / (40 * 128), a.alpha)
    res = tune(step, steps=a.steps, log=log)
    res.update(nbox=a.nbox, seed=a.seed, rcut=a.rcut, alpha=a.alpha, n=step.n)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
