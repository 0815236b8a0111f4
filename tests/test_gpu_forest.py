"""Batching: a forest of independent boxes in one node array, walked by one
persistent launch, gives each box exactly the forces of its own tree."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03567_amd.g4hip as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context()


SIZES = [4001, 20000, 777, 12345, 65]


def sr(n):
    scale = (128 ** 3 / n) ** (1.0 / 3.0)
    rs = 1.25 / 256 * scale
    return dict(r_s=rs, r_cut=4.5 * rs, eps0=scale / (40 * 128))


@pytest.fixture(scope="module")
def forest(g, ctx):
    boxes = [workloads.clustered_box(n, seed=900 + k, nhalo=max(2, n // 400), conc_spread=3.0)
             for k, n in enumerate(SIZES)]
    pos = np.concatenate([b.pos for b in boxes])
    m32 = np.concatenate([b.mass for b in boxes]).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(SIZES)]).astype(np.int64)
    tp = g.tree_params(True, 1.0, leaf_max=8)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(pos).cuda(), tp)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    f = g.g4_build_forest(ctx, off, p, tp)
    g.g4_compute_multipoles(ctx, f, 3)
    return boxes, off, f, m32, x, y, z, tp


def st3(o):
    return np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)


def single(g, ctx, x, y, z, m32, lo, hi, tp):
    p = g.particles(x[lo:hi].contiguous(), y[lo:hi].contiguous(), z[lo:hi].contiguous(),
                    torch.from_numpy(m32[lo:hi].copy()).cuda())
    t = g.g4_build_tree(ctx, p, tp)
    g.g4_compute_multipoles(ctx, t, 3)
    return t


@pytest.mark.parametrize("criterion,group", [(0, 64), (1, 64), (1, 32)])
def test_forest_equals_separate_trees(g, ctx, forest, criterion, group):
    boxes, off, f, m32, x, y, z, tp = forest
    kw = sr(20000)
    wp = g.walk_params(kernel=1, criterion=criterion, theta=0.7, alpha=0.005, theta_seed=0.7, group_size=group, **kw)
    out = st3(g.g4_treepm_shortrange(ctx, f, wp))
    for b in range(len(SIZES)):
        t = single(g, ctx, x, y, z, m32, off[b], off[b + 1], tp)
        ref = st3(g.g4_treepm_shortrange(ctx, t, wp))
        assert np.array_equal(out[off[b]:off[b + 1]], ref), f"box {b}"


def test_forest_node_sets_and_oracle_parity(g, ctx, forest):
    boxes, off, f, m32, x, y, z, tp = forest
    kw = sr(20000)
    ex = g.g4_tree_export(ctx, f, moments=False)
    lev, cnt = ex["level"].cpu().numpy(), ex["count"].cpu().numpy()
    assert np.sum(lev == 0) == len(SIZES)
    assert sorted(cnt[lev == 0].tolist()) == sorted(SIZES)
    wp = g.walk_params(kernel=1, criterion=0, theta=0.5, **kw)
    out = st3(g.g4_treepm_shortrange(ctx, f, wp))
    for b in (0, 1, 3):
        ps = boxes[b]
        st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
        ot = oracle.Tree(X, Y, Z, m32[off[b]:off[b + 1]].astype(np.float64), True, 1.0, 8)
        acc, _, _ = ot.walk(kernel=1, criterion=0, theta=0.5, nthreads=16, **kw)
        e = workloads.relative_errors(out[off[b]:off[b + 1]], acc)
        assert np.median(e) <= 1e-5 and np.percentile(e, 99.9) <= 1e-3, (b, np.median(e), e.max())


def test_forest_fmm_equals_separate(g, ctx, forest):
    """Sorted-list mode: bitwise equal to the boxes done one by one; atomic-sum
    mode: equal to round-off."""
    boxes, off, f, m32, x, y, z, tp = forest
    kw = sr(20000)
    for det in (1, 0):
        fp = g.fmm_params(kernel=1, theta=0.5, deterministic=det, **kw)
        out = st3(g.g4_fmm_force(ctx, f, fp))
        for b in (1, 2):
            t = single(g, ctx, x, y, z, m32, off[b], off[b + 1], tp)
            ref = st3(g.g4_fmm_force(ctx, t, fp))
            if det:
                assert np.array_equal(out[off[b]:off[b + 1]], ref), f"box {b}"
            else:
                e = workloads.relative_errors(out[off[b]:off[b + 1]], ref)
                assert np.median(e) <= 1e-6 and e.max() <= 1e-3, (b, np.median(e), e.max())


def test_forest_full_size_sampled_oracle_parity(g, ctx):
    """The 64-box forest at its real size (N log-uniform in [32768, 1048576],
    seeds 3000+b, concentration spread x3; about 15 M particles), walked in one
    persistent launch with the relative TreePM criterion at R_cut = 7 r_s,
    leaf 24: for 12 random targets per box the GPU forces equal the FP64
    oracle's at identical decisions (the oracle's own pre-walk |a| is given
    to the GPU for those targets)."""
    boxes = workloads.forest(64, seed=3000)
    sizes = [b.pos.shape[0] for b in boxes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    r_s, eps0 = 1.25 / 256, 1.0 / (40 * 128)
    kw = dict(r_s=r_s, r_cut=7 * r_s, eps0=eps0)
    B, alpha = 24, 0.001
    pos = np.concatenate([b.pos for b in boxes])
    m32 = np.concatenate([b.mass for b in boxes]).astype(np.float32)
    tp = g.tree_params(True, 1.0, leaf_max=B)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(pos).cuda(), tp)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    f = g.g4_build_forest(ctx, off, p, tp)
    g.g4_compute_multipoles(ctx, f, 3)
    gpre = g.g4_treepm_shortrange(ctx, f, g.walk_params(kernel=1, criterion=0, theta=0.7, **kw), want_amag=True)
    seed = gpre["amag"].clone()
    tgs, accs = [], []
    for b, ps in enumerate(boxes):
        st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
        ot = oracle.Tree(X, Y, Z, m32[off[b]:off[b + 1]].astype(np.float64), True, 1.0, B, nthreads=16)
        ot.compute_moments(nthreads=16)
        tg = workloads.sample_indices(sizes[b], 12, seed=700 + b)
        a0, _, _ = ot.walk(kernel=1, criterion=0, theta=0.7, targets=tg, nthreads=16, want_pot=False, **kw)
        s = np.zeros(sizes[b])
        s[tg] = np.linalg.norm(a0, axis=1)
        acc, _, cnt = ot.walk(kernel=1, criterion=1, alpha=alpha, aseed=s, targets=tg, nthreads=16, want_pot=False,
                              **kw)
        seed[off[b] + torch.from_numpy(tg).cuda()] = torch.from_numpy(s[tg].astype(np.float32)).cuda()
        tgs.append(tg + off[b])
        accs.append(acc)
        del ot
    tg = np.concatenate(tgs)
    ref = np.concatenate(accs)
    out = g.g4_treepm_shortrange(ctx, f, g.walk_params(kernel=1, criterion=1, alpha=alpha, a_seed=seed, **kw))
    a = st3(out)[tg]
    e = workloads.relative_errors(a, ref)
    print(f"forest {off[-1]} particles: median {np.median(e):.2e} p99.9 {np.percentile(e, 99.9):.2e}")
    assert np.median(e) <= 1e-5 and np.percentile(e, 99.9) <= 1e-3
