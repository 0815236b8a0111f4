"""Parity of the learned-seed kernels (features, forward, gradient, Adam) with the
FP64 oracle, given the same BF16-rounded weights and FP32 inputs."""
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


def random_weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    w = torch.from_numpy(rng.normal(scale=scale, size=oracle.NPARAM).astype(np.float32)).to(torch.bfloat16)
    return w.cuda(), w.double().numpy()


# leaf size 40: sources in more than one batch of the per-particle loop, and leaves
# beyond the register-staged moments path
@pytest.mark.parametrize("B", [8, 40])
def test_features_parity(g, ctx, B):
    ps = workloads.clustered_box(20001, seed=31, nhalo=40)
    tp = g.tree_params(True, 1.0, leaf_max=B)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(ps.pos).cuda(), tp)
    m32 = ps.mass.astype(np.float32)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    tree = g.g4_build_tree(ctx, p, tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    kw = dict(r_s=0.02, eps0=1.0 / (40 * 27))
    wp = g.walk_params(kernel=1, **kw)
    f = g.g4_mlp_features(ctx, tree, wp).cpu().numpy()
    st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    ot = oracle.Tree(X, Y, Z, m32.astype(np.float64), True, 1.0, B)
    ref = ot.features(kernel=1, **kw)
    np.testing.assert_allclose(f[:, :7], ref[:, :7], rtol=0, atol=2e-5)
    # near-field force feature: FP32 pair sums with the node centre of mass on the integer grid
    np.testing.assert_allclose(f[:, 7], ref[:, 7], rtol=0, atol=2e-4)
    # standardisation in the same call
    mu = ref.mean(0).astype(np.float32)
    inv = (1.0 / (ref.std(0) + 1e-6)).astype(np.float32)
    norm = torch.from_numpy(np.concatenate([mu, inv])).cuda()
    fn = g.g4_mlp_features(ctx, tree, wp, norm).cpu().numpy()
    np.testing.assert_allclose(fn, (f - mu) * inv, rtol=0, atol=1e-4)


@pytest.mark.parametrize("n", [1, 1000, 4097])
def test_forward_parity(g, ctx, n):
    w, wd = random_weights(7)
    rng = np.random.default_rng(n)
    feat = rng.normal(size=(n, 8)).astype(np.float32)
    y = g.g4_mlp_forward(ctx, w, torch.from_numpy(feat).cuda()).cpu().numpy()
    ref = oracle.mlp_forward(wd, feat.astype(np.float64))
    np.testing.assert_allclose(y, ref, rtol=0, atol=2e-5 * max(1.0, np.abs(ref).max()))
    a = g.g4_mlp_forward(ctx, w, torch.from_numpy(feat).cuda(), shift=-0.25, mode=1).cpu().numpy()
    np.testing.assert_allclose(a, 10.0 ** (ref - 0.25), rtol=1e-4)


@pytest.mark.parametrize("n,tau", [(1, 0.0), (300, 0.0), (5000, 0.0), (5000, 0.25)])
def test_gradient_parity(g, ctx, n, tau):
    """GPU backpropagation against the FP64 oracle's gradient (itself pinned by
    finite differences on the CPU)."""
    w, wd = random_weights(11)
    rng = np.random.default_rng(100 + n)
    feat = rng.normal(size=(n, 8)).astype(np.float32)
    tgt = rng.normal(size=n).astype(np.float32)
    grad, loss = g.g4_mlp_grad(ctx, w, torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda(), tau)
    lref, gref = oracle.mlp_loss_grad(wd, feat.astype(np.float64), tgt.astype(np.float64), tau)
    assert loss.item() == pytest.approx(lref, rel=1e-4)
    gg = grad.cpu().numpy()
    scale = np.abs(gref).max()
    assert np.abs(gg - gref).max() <= 1e-4 * scale
    for sl in (slice(0, 512), slice(512, 576), slice(576, 4672), slice(4672, 4736), slice(4736, 4801)):
        assert np.abs(gg[sl] - gref[sl]).max() <= 1e-4 * max(np.abs(gref[sl]).max(), 1e-3 * scale)


def test_adam_parity(g, ctx):
    rng = np.random.default_rng(3)
    master = rng.normal(scale=0.2, size=oracle.NPARAM).astype(np.float32)
    m = rng.normal(scale=1e-3, size=oracle.NPARAM).astype(np.float32)
    v = np.abs(rng.normal(scale=1e-5, size=oracle.NPARAM)).astype(np.float32)
    grad = rng.normal(scale=1e-2, size=oracle.NPARAM).astype(np.float32)
    dev = lambda a: torch.from_numpy(a.copy()).cuda()
    wb = torch.empty(oracle.NPARAM, dtype=torch.bfloat16, device="cuda")
    tm, tmm, tv = dev(master), dev(m), dev(v)
    g.g4_mlp_adam(ctx, wb, tm, tmm, tv, dev(grad), lr=1e-3, step=5)
    wd, md, vd = master.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    oracle.adam(wd, grad.astype(np.float64), md, vd, lr=1e-3, step=5)
    np.testing.assert_allclose(tm.cpu().numpy(), wd, rtol=1e-5, atol=1e-7)
    # m = b1 m + (1 - b1) g in FP32: terms of ~1e-3 round at ~1e-10, and cancel for small m
    np.testing.assert_allclose(tmm.cpu().numpy(), md, rtol=1e-5, atol=2e-9)
    # the BF16 copy is the round-to-nearest-even of the FP32 master weights
    assert torch.equal(wb.cpu(), tm.cpu().to(torch.bfloat16))


def test_training_reduces_loss(g, ctx):
    """A few hundred Adam steps on a smooth synthetic target cut the loss."""
    rng = np.random.default_rng(9)
    n = 8192
    feat = rng.normal(size=(n, 8)).astype(np.float32)
    tgt = (np.sin(feat[:, 0]) + 0.5 * feat[:, 1] * feat[:, 2] - 0.3 * feat[:, 3] ** 2).astype(np.float32)
    w, _ = random_weights(5, scale=0.1)
    master = w.float().clone()
    state = torch.zeros(2 * oracle.NPARAM, dtype=torch.float32, device="cuda")
    grad = torch.empty(oracle.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    f, t = torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda()
    losses = []
    for step in range(1, 401):
        g.g4_mlp_train_step(ctx, w, master, state, grad, f, t, 3e-3, step, loss)
        if step in (1, 400):
            losses.append(loss.item())
    assert losses[1] < 0.2 * losses[0]
