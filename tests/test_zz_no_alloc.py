"""g4_fmm_force_noalloc (static device scratch, no workspace argument) against
g4_fmm_force (caller's workspace) through the C ABI: bitwise in the
sorted-list mode, to round-off in the atomic-sum mode, on two calls in a row
with the second on a smaller tree (the scratch keeps the first call's
contents), and a tree too large for the scratch is refused on the host."""
import numpy as np
import pytest
import torch

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


def _case(g, ctx, n, seed):
    ps = workloads.clustered_box(n, seed=seed, nhalo=max(4, n // 500))
    tp = g.tree_params(True, 1.0, leaf_max=16)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(ps.pos).cuda(), tp)
    p = g.particles(x, y, z, torch.from_numpy(ps.mass.astype(np.float32)).cuda())
    tree = g.g4_build_tree(ctx, p, tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    scale = (128 ** 3 / n) ** (1.0 / 3.0)
    r_s = 1.25 / 256 * scale
    return tree, dict(r_s=r_s, r_cut=4.5 * r_s, eps0=scale / (40 * 128))


def _a(o):
    return np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)


# the sorted-list mode needs ~7 kB of lists per particle, the atomic-sum mode ~0.5 kB
@pytest.mark.parametrize("det,sizes", [(1, (6000, 2501)), (0, (60000, 7001))])
def test_noalloc_fmm_matches_workspace_fmm(g, ctx, det, sizes):
    for n, seed in zip(sizes, (31, 32)):  # second call on a smaller tree
        tree, kw = _case(g, ctx, n, seed)
        fp = g.fmm_params(kernel=1, theta=0.5, deterministic=det, **kw)
        ref = g.g4_fmm_force(ctx, tree, fp, want_pot=True, want_stats=True)
        got = g.g4_fmm_force_noalloc(ctx, tree, fp, want_pot=True, want_stats=True)
        a_ref, a_got = _a(ref), _a(got)
        for k in ("n_pp", "n_pn", "n_nn"):
            assert got["stats"][k] == ref["stats"][k], k
        if det:
            assert np.array_equal(a_got, a_ref) and torch.equal(got["pot"], ref["pot"]), n
        else:
            e = workloads.relative_errors(a_got, a_ref)
            assert np.median(e) <= 1e-6 and np.percentile(e, 99.9) <= 1e-4, (n, np.median(e), e.max())
            dp = (got["pot"] - ref["pot"]).abs() / ref["pot"].abs().clamp_min(1e-30)
            assert float(dp.max()) <= 1e-4


def test_noalloc_fmm_rejects_tree_beyond_scratch(g, ctx):
    tree, kw = _case(g, ctx, 400000, 33)
    fp = g.fmm_params(kernel=1, theta=0.5, **kw)
    with pytest.raises(g.G4Error) as e:
        g.g4_fmm_force_noalloc(ctx, tree, fp)
    assert e.value.code == g.G4_EINVAL and "static FMM scratch" in str(e.value)
