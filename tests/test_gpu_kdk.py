"""The hierarchical time integration driver (g4_kdk_step) through the C ABI:
with FP64 direct-sum forces it must retrace the oracle's hierarchical steps
(same splits, same force count, positions and velocities to round-off); with
the FMM it must conserve momentum to FP32 round-off (every force is sourced by
the set it acts on); the tree-walk solver follows the direct-sum trajectory
to its force error."""
import numpy as np
import pytest
import torch

import workloads
from oracle import kdk

pytestmark = pytest.mark.gpu

ROOT = (np.array([-40.0, -40.0, -40.0]), 80.0)


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03567_amd.g4hip as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context()


def _plummer(n, seed):
    ps = workloads.plummer(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    vel = 0.3 * rng.normal(size=(n, 3))
    vel -= (ps.mass[:, None] * vel).sum(0) / ps.mass.sum()
    return ps.pos.copy(), vel, ps.mass.astype(np.float32).astype(np.float64)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def test_kdk_direct_matches_oracle(g, ctx):
    n, eps, eta, dt = 400, 0.02, 0.025, 0.05
    pos, vel, m = _plummer(n, 21)
    tp = g.tree_params(False, ROOT[1], tuple(ROOT[0]), leaf_max=8)
    kp = g.kdk_params(0, tp, eta, eps, max_level=12, wp=g.walk_params(kernel=0, eps0=eps))
    P, V, M = _dev(pos), _dev(vel), _dev(m, torch.float32)
    force = kdk.direct_force(m, eps0=eps, root=ROOT)
    idx = np.arange(n)
    a = force(idx, pos)
    acc = None
    for step in range(3):
        c = kdk.Counter()
        a = kdk.hierarchical_step(idx, dt, a, pos, vel, force, eta, eps, max_level=12, count=c)
        acc, st, ws = g.g4_kdk_step(ctx, kp, P, V, M, dt, acc=acc)
        assert st["force_evals"] - (n if step == 0 else 0) == c.evals, (st, c.evals)
        assert st["deepest_level"] >= 2
    np.testing.assert_allclose(P.cpu().numpy(), pos, rtol=0, atol=1e-9)
    np.testing.assert_allclose(V.cpu().numpy(), vel, rtol=1e-9, atol=1e-9 * np.abs(vel).max())
    ga = np.stack([t.cpu().numpy() for t in acc], 1)
    np.testing.assert_allclose(ga, a, rtol=1e-9, atol=1e-9 * np.abs(a).max())


def test_kdk_fmm_conserves_momentum(g, ctx):
    n = 30000
    ps = workloads.clustered_box(n, seed=23, nhalo=40)
    scale = (128 ** 3 / n) ** (1 / 3)
    r_s, eps = 1.25 / 256 * scale, scale / (40 * 128)
    tp = g.tree_params(True, 1.0, leaf_max=16)
    fp = g.fmm_params(kernel=1, theta=0.5, r_s=r_s, r_cut=4.5 * r_s, eps0=eps)
    kp = g.kdk_params(2, tp, 0.025, eps, max_level=8, fp=fp)
    rng = np.random.default_rng(24)
    m = ps.mass.astype(np.float32)
    vel = 0.05 * rng.normal(size=(n, 3))
    P, V, M = _dev(ps.pos), _dev(vel), _dev(m, torch.float32)
    p0 = (m[:, None].astype(np.float64) * vel).sum(0)
    acc = None
    for _ in range(2):
        acc, st, ws = g.g4_kdk_step(ctx, kp, P, V, M, 0.002, acc=acc)
    v = V.cpu().numpy()
    dp = np.abs((m[:, None] * v).sum(0) - p0).max()
    print("fmm kdk: levels", st["deepest_level"], "force evals", st["force_evals"], "momentum drift", dp)
    assert st["deepest_level"] >= 2
    assert dp <= 1e-6 * (m[:, None] * np.abs(v)).sum()
    x = P.cpu().numpy()
    assert np.all((x >= 0) & (x < 1.0))


def test_kdk_tree_walk_follows_direct(g, ctx):
    n, eps, eta, dt = 2000, 0.02, 0.025, 0.05
    pos, vel, m = _plummer(n, 31)
    tp = g.tree_params(False, ROOT[1], tuple(ROOT[0]), leaf_max=8)
    out = {}
    for solver, wp in ((0, g.walk_params(kernel=0, eps0=eps)),
                       (1, g.walk_params(kernel=0, eps0=eps, criterion=1, alpha=0.0005, theta_seed=0.7))):
        kp = g.kdk_params(solver, tp, eta, eps, max_level=12, wp=wp)
        P, V, M = _dev(pos), _dev(vel), _dev(m, torch.float32)
        acc = None
        for _ in range(2):
            acc, st, ws = g.g4_kdk_step(ctx, kp, P, V, M, dt, acc=acc)
        out[solver] = (P.cpu().numpy(), V.cpu().numpy())
    dv = np.linalg.norm(out[1][1] - out[0][1], axis=1) / np.linalg.norm(out[0][1], axis=1)
    print("tree vs direct velocity difference: median", np.median(dv), "p99", np.percentile(dv, 99))
    assert np.median(dv) < 1e-3
