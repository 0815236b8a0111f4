"""The long-range (PM) force through the C ABI: parity with the FP64 oracle's
PM at the same mesh (element by element, small meshes and the 256^3 mesh of
the 128^3 configuration), zero net force, the accumulate mode, and the total
TreePM force (short-range walk + PM) against the exact periodic force of the
Ewald decomposition on a small box.

Tolerance of the PM parity (derived from the arithmetic): the mesh is FP32,
the transforms are ng-point radix-2 FFTs (about log2 ng roundings of ~6e-8
per value) and the gradient takes differences of neighbouring potentials, so
per-particle long-range forces agree with the FP64 oracle to ~1e-5 of their
own size; the bar is median <= 2e-5 and 99.9th percentile <= 1e-3.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import pm as opm

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


def build(g, ctx, ps, B=16):
    tp = g.tree_params(True, 1.0, leaf_max=B)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(ps.pos).cuda(), tp)
    m32 = ps.mass.astype(np.float32)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    tree = g.g4_build_tree(ctx, p, tp)
    X, Y, Z = (v.cpu().numpy().view(np.uint32) for v in (x, y, z))
    return tree, p, tp, m32, X, Y, Z


def st3(o):
    return np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)


def oracle_pm(X, Y, Z, m, ng, r_s, want_pot=False):
    c, f = opm.cic_cells_int(X, Y, Z, ng)
    return opm.pm_long_range(c, f, m.astype(np.float64), ng, 1.0, r_s, want_pot=want_pot)


def check(a, ref, label, med=2e-5, p999=1e-3):
    e = workloads.relative_errors(a, ref)
    msg = f"{label}: median {np.median(e):.2e} p99.9 {np.percentile(e, 99.9):.2e} max {e.max():.2e}"
    print(msg)
    assert np.median(e) <= med and np.percentile(e, 99.9) <= p999, msg


@pytest.mark.parametrize("n,ng", [(20000, 32), (20000, 64), (3001, 16), (70000, 128)])
def test_pm_parity_with_oracle(g, ctx, n, ng):
    ps = workloads.clustered_box(n, seed=50 + ng, nhalo=max(4, n // 400))
    tree, p, tp, m32, X, Y, Z = build(g, ctx, ps)
    r_s = 1.25 / ng
    out = g.g4_pm_longrange(ctx, tree, g.pm_params(ng, r_s), want_pot=True)
    ref, pref = oracle_pm(X, Y, Z, m32, ng, r_s, want_pot=True)
    check(st3(out), ref, f"pm n={n} ng={ng}")
    dp = np.abs(out["pot"].cpu().numpy() - pref) / np.abs(pref).max()
    assert np.median(dp) <= 2e-6 and dp.max() <= 1e-4
    a = st3(out)
    net = np.abs((m32[:, None].astype(np.float64) * a).sum(0)).max() / (m32[:, None] * np.abs(a)).sum()
    assert net <= 1e-5, net


def test_pm_full_mesh_parity_128cube(g, ctx):
    """The clustered 128^3 box with the configuration's 256^3 mesh (r_s = 1.25/256)."""
    n, ng = 128 ** 3, 256
    ps = workloads.clustered_box(n, seed=2)
    tree, p, tp, m32, X, Y, Z = build(g, ctx, ps, B=24)
    out = g.g4_pm_longrange(ctx, tree, g.pm_params(ng, 1.25 / 256))
    ref = oracle_pm(X, Y, Z, m32, ng, 1.25 / 256)
    check(st3(out), ref, "pm 128^3 ng=256")


def test_pm_accumulates_onto_the_walk(g, ctx):
    ps = workloads.clustered_box(30000, seed=61, nhalo=60)
    tree, p, tp, m32, X, Y, Z = build(g, ctx, ps)
    g.g4_compute_multipoles(ctx, tree, 3)
    ng = 32
    r_s = 1.25 / ng
    wp = g.walk_params(kernel=1, criterion=0, theta=0.5, r_s=r_s, r_cut=4.5 * r_s)
    w = g.g4_treepm_shortrange(ctx, tree, wp)
    sr = st3(w)
    lr = st3(g.g4_pm_longrange(ctx, tree, g.pm_params(ng, r_s)))
    tot = g.g4_pm_longrange(ctx, tree, g.pm_params(ng, r_s), accumulate=True, out=(w["ax"], w["ay"], w["az"], None))
    # the mass assignment sums with float atomics, so two PM calls agree to FP32 round-off only
    e = workloads.relative_errors(st3(tot) - sr, lr)
    assert np.median(e) <= 1e-6 and e.max() <= 1e-4, (np.median(e), e.max())


def test_total_treepm_force_against_exact_ewald(g, ctx):
    """Short-range walk (R_cut = 4.5 r_s, relative criterion) + PM against the
    exact periodic force (short-range q = 0 direct sum + exact k-space sum of
    the Ewald decomposition): the total force error is set by the PM and the
    cut-off at the matching scale, as in the paper's TreePM force-law figures
    (max errors of order 1e-2 at R_cut 4.5); and the GPU total equals the
    oracle's own TreePM total (walk + PM) at identical decisions."""
    n, ng = 2000, 32
    ps = workloads.clustered_box(n, seed=71, nhalo=6)
    tree, p, tp, m32, X, Y, Z = build(g, ctx, ps, B=8)
    g.g4_compute_multipoles(ctx, tree, 3)
    r_s = 1.25 / ng
    kw = dict(kernel=1, r_s=r_s, r_cut=4.5 * r_s, eps0=1.0 / (40 * 12.6))
    tg = workloads.sample_indices(n, 400, seed=3)
    # oracle: seed walk, relative walk, PM; the GPU gets the oracle's seeds
    ot = oracle.Tree(X, Y, Z, m32.astype(np.float64), True, 1.0, 8)
    a0, _, _ = ot.walk(criterion=0, theta=0.7, **kw)
    seed = np.linalg.norm(a0, axis=1)
    osr, _, _ = ot.walk(criterion=1, alpha=0.002, aseed=seed, **kw)
    olr = oracle_pm(X, Y, Z, m32, ng, r_s)
    wp = g.walk_params(criterion=1, alpha=0.002, a_seed=torch.from_numpy(seed.astype(np.float32)).cuda(), **kw)
    w = g.g4_treepm_shortrange(ctx, tree, wp)
    tot = st3(g.g4_pm_longrange(ctx, tree, g.pm_params(ng, r_s), accumulate=True,
                                out=(w["ax"], w["ay"], w["az"], None)))
    check(tot, osr + olr, "total treepm vs oracle treepm")
    # exact periodic force: untruncated short-range sum + exact k-space sum
    pos = np.stack([X, Y, Z], 1).astype(np.float64) * 2.0 ** -32
    sr_ex, _ = oracle.direct(X, Y, Z, m32.astype(np.float64), 2.0 ** -32, kernel=1, eps0=kw["eps0"], r_s=r_s,
                             r_cut=np.inf, targets=tg, nthreads=8)
    lr_ex, _ = opm.ewald_long_range(pos[tg], pos, m32.astype(np.float64), 1.0, r_s, kcut=5.0)
    e = workloads.relative_errors(tot[tg], sr_ex + lr_ex)
    print(f"total TreePM vs exact Ewald: median {np.median(e):.2e} p99 {np.percentile(e, 99):.2e} max {e.max():.2e}")
    assert np.median(e) < 5e-3 and np.percentile(e, 99) < 3e-2
