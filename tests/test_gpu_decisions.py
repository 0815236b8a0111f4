"""The constructed decision cases of the oracle's pins, run through the HIP
walk and FMM: each kernel must take the paper's decision for the one node (or
node pair) in question, not merely agree with the oracle on random inputs.

The exclusion test and the FMM touching test are exact integer decisions on
both sides.  The relative criterion, the softening edge and the r_cut drop are
evaluated in FP32 on the GPU, so their thresholds are probed at 1e-4 instead
of the oracle's 1e-7.
"""
import math

import numpy as np
import pytest
import torch

from test_oracle_decisions import ACCEPTED, DROPPED, OPENED, _fmm_relative_thresholds, fmm_positions, walk_positions

pytestmark = pytest.mark.gpu
MARGIN = 1e-4


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03567_amd.g4hip as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context()


def _tree(g, ctx, X, Y, Z, m, B):
    dev = ctx.device
    xs = [torch.from_numpy(v.astype(np.uint32).view(np.int32)).to(dev) for v in (X, Y, Z)]
    p = g.particles(*xs, torch.from_numpy(m.astype(np.float32)).to(dev))
    tp = g.tree_params(True, 1.0, leaf_max=B)
    tree = g.g4_build_tree(ctx, p, tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    return tree


def _counts(g, ctx, lev_n, offset, aseed=None, **kw):
    X, Y, Z, m, l, r = walk_positions(lev_n, offset)
    tree = _tree(g, ctx, X, Y, Z, m, 2)
    a = None if aseed is None else torch.tensor(aseed, dtype=torch.float32, device=ctx.device)
    wp = g.walk_params(G=1.0, a_seed=a, **kw)
    out = g.g4_tree_force(ctx, tree, wp, want_counts=True)
    c = out["counts"].cpu().numpy()
    return tuple(int(v) for v in c[2])


def _lr(lev_n, offset):
    _, _, _, _, l, r = walk_positions(lev_n, offset)
    return l, r


@pytest.mark.parametrize("lev_n", [4, 9])
def test_gpu_exclusion_zone_is_cube_of_side_2l(g, ctx, lev_n):
    ln = 1 << (32 - lev_n)
    geo = dict(criterion=0, theta=1e6, eps0=0.0, exclusion=1)
    assert _counts(g, ctx, lev_n, (ln - 1, 0, 0), **geo) == OPENED
    assert _counts(g, ctx, lev_n, (ln, 0, 0), **geo) == ACCEPTED
    assert _counts(g, ctx, lev_n, (ln - 1, ln - 1, ln - 1), **geo) == OPENED
    assert _counts(g, ctx, lev_n, (ln - 1, ln - 1, ln), **geo) == ACCEPTED


@pytest.mark.parametrize("order", [3, 2])
def test_gpu_relative_criterion_threshold_and_exponent(g, ctx, order):
    ln = 1 << 28
    off = (ln + ln // 4, 0, 0)
    l, r = _lr(4, off)
    A = 0.37
    a_crit = l ** order / (A * r ** (order + 2))
    kw = dict(criterion=1, order=order, eps0=0.0, exclusion=1, aseed=[1.0, 1.0, A])
    assert _counts(g, ctx, 4, off, alpha=a_crit * (1 + MARGIN), **kw) == ACCEPTED
    assert _counts(g, ctx, 4, off, alpha=a_crit * (1 - MARGIN), **kw) == OPENED


def test_gpu_relative_criterion_scales_as_l_cubed(g, ctx):
    d = (1 << 28) + (1 << 26)
    kw = dict(criterion=1, order=3, eps0=0.0, exclusion=0, aseed=[1.0, 1.0, 1.0])
    for lev_n in (4, 3):
        l, r = _lr(lev_n, (d, 0, 0))
        crit = l ** 3 / r ** 5
        assert _counts(g, ctx, lev_n, (d, 0, 0), alpha=crit * (1 + MARGIN), **kw) == ACCEPTED
        assert _counts(g, ctx, lev_n, (d, 0, 0), alpha=crit * (1 - MARGIN), **kw) == OPENED


def test_gpu_nodes_closer_than_softening_edge_are_opened(g, ctx):
    ln = 1 << 28
    off = (ln + ln // 4, 0, 0)
    l, r = _lr(4, off)
    geo = dict(criterion=0, theta=1e6, exclusion=1)
    assert _counts(g, ctx, 4, off, eps0=r / 2.8 * (1 + MARGIN), **geo) == OPENED
    assert _counts(g, ctx, 4, off, eps0=r / 2.8 * (1 - MARGIN), **geo) == ACCEPTED


def test_gpu_treepm_drops_nodes_by_nearest_edge_distance(g, ctx):
    ln = 1 << 28
    kw = dict(kernel=1, r_s=0.01, criterion=0, theta=1e6, eps0=0.0, exclusion=1)
    off = (ln + ln // 4, 0, 0)
    l, r = _lr(4, off)
    e = 0.75 * l
    assert _counts(g, ctx, 4, off, r_cut=e * (1 + MARGIN), **kw) == ACCEPTED
    assert _counts(g, ctx, 4, off, r_cut=e * (1 - MARGIN), **kw) == DROPPED
    off = (ln + ln // 4, ln + ln // 4, 0)
    e2 = math.sqrt(2.0) * 0.75 * l
    assert _counts(g, ctx, 4, off, r_cut=e2 * (1 + MARGIN), **kw) == ACCEPTED
    assert _counts(g, ctx, 4, off, r_cut=0.9 * e2, **kw) == DROPPED


@pytest.mark.parametrize("det", [0, 1])
@pytest.mark.parametrize("cells,expect", [
    ([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)], (3, 0, 3)),
    ([(0, 0, 0), (1, 1, 1)], (1, 0, 0)),
    ([(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 3, 3)], (3, 0, 3)),
])
def test_gpu_fmm_touching_cells_never_interact(g, ctx, cells, expect, det):
    X, Y, Z, m = fmm_positions(cells)
    tree = _tree(g, ctx, X, Y, Z, m, 1)
    fp = g.fmm_params(kernel=0, theta=1e6, eps0=0.0, deterministic=det)
    out = g.g4_fmm_force(ctx, tree, fp, want_stats=True)
    s = out["stats"]
    assert (s["n_pp"], s["n_pn"], s["n_nn"]) == expect


@pytest.mark.parametrize("det", [0, 1])
def test_gpu_fmm_relative_criterion_threshold(g, ctx, det):
    """The oracle's four-leaf line with unequal masses and seeds: each
    non-touching pair switches to a node-node interaction as alpha passes its
    threshold M_max l_max^2 / (|a|_min r^4), probed at 1 +- 1e-4."""
    import oracle
    X, Y, Z, _ = fmm_positions([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    m = np.array([1.0, 2.0, 3.0, 0.5])
    aseed = np.array([5.0, 0.7, 3.0, 2.0], np.float32)
    tree = _tree(g, ctx, X, Y, Z, m, 1)
    thr = sorted(_fmm_relative_thresholds(oracle.Tree(X, Y, Z, m, True, 1.0, 1), m, aseed.astype(np.float64)).values())
    sd = torch.from_numpy(aseed).cuda()
    for k, a in enumerate(thr):
        for f, want in ((1 + MARGIN, k + 1), (1 - MARGIN, k)):
            fp = g.fmm_params(kernel=0, eps0=0.0, deterministic=det, criterion=1, alpha=a * f, a_seed=sd)
            s = g.g4_fmm_force(ctx, tree, fp, want_stats=True)["stats"]
            assert s["n_nn"] == want, (k, f, s["n_nn"])


def test_gpu_stats_phase_times(g, ctx):
    """g4_stats carries the hipEvent durations of the build, the moments, the
    seed (pre-walk) and the walk; each is positive and together they fit in
    the host's wall time around the same calls.  A geometric call has no seed
    phase, and a FMM call reports its whole duration as t_walk."""
    import time

    import workloads
    ps = workloads.clustered_box(200000, seed=5, nhalo=50)
    pos = torch.from_numpy(ps.pos).to(ctx.device)
    m = torch.from_numpy(ps.mass.astype(np.float32)).to(ctx.device)
    tp = g.tree_params(True, 1.0, leaf_max=16)
    n = ps.pos.shape[0]
    kw = dict(kernel=1, r_s=1.25 / 256 * (128 ** 3 / n) ** (1 / 3), eps0=0.0)
    kw["r_cut"] = 4.5 * kw["r_s"]
    x, y, z = g.g4_quantize(ctx, pos, tp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = g.g4_build_tree(ctx, g.particles(x, y, z, m), tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    out = g.g4_tree_force(ctx, tree, g.walk_params(criterion=1, alpha=0.005, **kw), want_stats=True)
    wall = time.perf_counter() - t0
    s = out["stats"]
    ts = [s["t_build"], s["t_moments"], s["t_seed"], s["t_walk"]]
    print("phase times", ts, "wall", wall)
    assert all(t > 0 for t in ts) and sum(ts) <= wall
    s = g.g4_tree_force(ctx, tree, g.walk_params(criterion=0, theta=0.7, **kw), want_stats=True)["stats"]
    assert s["t_seed"] == 0.0 and s["t_walk"] > 0 and s["flags"] & 0xC == 0
    s = g.g4_fmm_force(ctx, tree, g.fmm_params(kernel=1, theta=0.5, r_s=kw["r_s"], r_cut=kw["r_cut"]),
                       want_stats=True)["stats"]
    assert s["t_walk"] > 0 and s["t_build"] > 0 and s["flags"] & 0xC == 0
