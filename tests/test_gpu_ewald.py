"""The periodic tree walk with the Ewald correction (kernel 2, Sec. "Periodic
boundary conditions") through the C ABI: the table of psi's derivatives
against the oracle's exact Ewald sums, its third-order Taylor lookup at
arbitrary offsets, the walk at identical decisions against the oracle's
periodic walk, theta -> 0 against the oracle's Ewald direct sum, and a lattice
whose exact forces vanish."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

NE = 32


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_03567_amd.g4hip as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context()


@pytest.fixture(scope="module")
def table(g, ctx):
    return g.EwaldTable(ctx, 1.0, NE)


def _idx(a, b, c):
    o = a + b + c
    return o * (o + 1) * (o + 2) // 6 + (b + c) * (b + c + 1) // 2 + c


def test_table_holds_the_ewald_derivatives(g, ctx, table):
    """Grid values of orders 0..3 equal the oracle's FP64 Ewald sums to FP32
    rounding; orders 4..6 equal central differences of the oracle's third
    derivatives."""
    tab = table.values().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(1)
    pts = [(0, 0, 0), (NE, NE, NE), (NE, 0, 0), (3, 17, 29)] + [tuple(rng.integers(0, NE + 1, 3)) for _ in range(12)]
    h = 0.5 / NE
    for (i, j, k) in pts:
        row = tab[(i * (NE + 1) + j) * (NE + 1) + k]
        x = np.array([i, j, k], float) * h
        D0, D1, D2, D3 = (a[0] for a in oracle.ewald_psi(x))
        assert abs(row[0] - D0) <= 1e-6 * abs(D0)
        for a in range(3):
            e = [0, 0, 0]; e[a] = 1
            assert abs(row[_idx(*e)] - D1[a]) <= 1e-6 * max(1.0, np.abs(D1).max())
            for b in range(3):
                e2 = list(e); e2[b] += 1
                assert abs(row[_idx(*e2)] - D2[a, b]) <= 1e-6 * max(1.0, np.abs(D2).max())
                for c in range(3):
                    e3 = list(e2); e3[c] += 1
                    assert abs(row[_idx(*e3)] - D3[a, b, c]) <= 1e-6 * max(1.0, np.abs(D3).max())
    # order 4 from differences of D3 (step 1e-4: error ~1e-7 of the scale)
    for (i, j, k) in pts[2:8]:
        row = tab[(i * (NE + 1) + j) * (NE + 1) + k]
        x = np.array([i, j, k], float) * h
        s = 1e-4
        for a in range(3):
            e = np.zeros(3); e[a] = s
            d3p = oracle.ewald_psi(x + e)[3][0]
            d3m = oracle.ewald_psi(x - e)[3][0]
            d4 = (d3p - d3m) / (2 * s)
            scale = max(1.0, np.abs(d4).max())
            for b in range(3):
                for c in range(3):
                    for d in range(3):
                        m = [0, 0, 0]
                        for q in (a, b, c, d):
                            m[q] += 1
                        assert abs(row[_idx(*m)] - d4[b, c, d]) <= 1e-5 * scale, (i, j, k, a, b, c, d)


def test_taylor_lookup_at_arbitrary_offsets(g, ctx, table):
    """psi and grad psi between grid points, in every octant and on the cell
    faces, against the oracle's exact sums: the third-order expansion with a
    grid of L/64 leaves less than ~2e-5 of the gradient's scale."""
    rng = np.random.default_rng(2)
    d = np.concatenate([rng.uniform(-0.5, 0.5, size=(150, 3)),
                        [[0.5, 0.5, 0.5], [-0.5, 0.2, 0.1], [1e-4, -2e-4, 3e-4], [0.0, 0.0, 0.0],
                         [0.49, -0.49, 0.013]]])
    psi, grad = g.g4_ewald_eval(ctx, table, torch.from_numpy(d).cuda())
    psi, grad = psi.cpu().numpy(), grad.cpu().numpy()
    D0, D1, _, _ = oracle.ewald_psi(d)
    perr = np.abs(psi - D0).max()
    gerr = np.abs(grad - D1).max(axis=1)
    print(f"psi max abs err {perr:.2e}; grad max abs err {gerr.max():.2e} (scale {np.abs(D1).max():.2f})")
    assert perr <= 2e-6 * abs(D0).max()
    assert np.all(gerr <= 2e-5 * max(1.0, np.abs(D1).max()))


def _case(g, ctx, n, seed, B=8):
    ps = workloads.clustered_box(n, seed=seed, nhalo=max(4, n // 300))
    tp = g.tree_params(True, 1.0, leaf_max=B)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(ps.pos).cuda(), tp)
    m32 = ps.mass.astype(np.float32)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    tree = g.g4_build_tree(ctx, p, tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    ot = oracle.Tree(X, Y, Z, m32.astype(np.float64), True, 1.0, B)
    ot.compute_moments()
    eps = (128 ** 3 / n) ** (1 / 3) / (40 * 128)
    return tree, ot, (X, Y, Z, m32), eps


def _stack(o):
    return np.stack([o["ax"].cpu().numpy(), o["ay"].cpu().numpy(), o["az"].cpu().numpy()], 1)


def _parity(a, ref, cg=None, co=None, label=""):
    err = workloads.relative_errors(a, ref)
    msg = f"{label}: median {np.median(err):.2e} p99.9 {np.percentile(err, 99.9):.2e} max {err.max():.2e}"
    if cg is not None:
        agree = np.mean(np.all(cg.astype(np.int64) == co, axis=1))
        msg += f" agreement {agree:.4f}"
        assert agree >= 0.999, msg
    print(msg)
    assert np.median(err) <= 1e-5 and np.percentile(err, 99.9) <= 1e-3, msg


@pytest.mark.parametrize("order", [3, 2])
def test_walk_parity_with_the_oracle(g, ctx, table, order):
    tree, ot, _, eps = _case(g, ctx, 2500, 41)
    wp = g.walk_params(kernel=2, criterion=0, theta=0.5, order=order, eps0=eps, ewald=table)
    out = g.g4_tree_force(ctx, tree, wp, want_pot=True, want_counts=True)
    acc, pot, cnt = ot.walk(kernel=2, criterion=0, theta=0.5, order=order, eps0=eps, nthreads=16)
    _parity(_stack(out), acc, out["counts"].cpu().numpy(), cnt, f"ewald geometric p={order}")
    perr = np.abs(out["pot"].cpu().numpy() - pot) / np.abs(pot)
    assert np.median(perr) < 1e-5, np.median(perr)
    seed = np.linalg.norm(acc, axis=1).astype(np.float32)
    wp = g.walk_params(kernel=2, criterion=1, alpha=0.002, order=order, eps0=eps,
                       a_seed=torch.from_numpy(seed).cuda(), ewald=table)
    out = g.g4_tree_force(ctx, tree, wp, want_counts=True)
    acc, _, cnt = ot.walk(kernel=2, criterion=1, alpha=0.002, order=order, eps0=eps, aseed=seed, nthreads=16)
    _parity(_stack(out), acc, out["counts"].cpu().numpy(), cnt, f"ewald relative p={order}")


def test_theta_to_zero_is_the_ewald_direct_sum(g, ctx, table):
    tree, ot, (X, Y, Z, m32), eps = _case(g, ctx, 500, 43)
    out = g.g4_tree_force(ctx, tree, g.walk_params(kernel=2, criterion=0, theta=1e-6, eps0=eps, ewald=table),
                          want_pot=True)
    ref, pot = oracle.direct(X, Y, Z, m32.astype(np.float64), 1.0 / 2 ** 32, kernel=2, eps0=eps, nthreads=16)
    err = workloads.relative_errors(_stack(out), ref)
    print(f"theta -> 0 vs Ewald direct sum: median {np.median(err):.2e} max {err.max():.2e}")
    assert np.median(err) <= 1e-5 and err.max() <= 1e-3
    assert np.median(np.abs(out["pot"].cpu().numpy() - pot) / np.abs(pot)) <= 1e-5


def test_lattice_feels_no_force(g, ctx, table):
    """Equal masses on a 4^3 lattice: the exact periodic forces vanish; the
    walk at theta -> 0 leaves FP32 round-off of the single-pair scale m/(L/4)^2."""
    gg = (np.arange(4) + 0.25) / 4
    pos = np.stack(np.meshgrid(gg, gg, gg, indexing="ij"), -1).reshape(-1, 3)
    m = np.full(64, 1.0 / 64, np.float32)
    tp = g.tree_params(True, 1.0, leaf_max=1)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(pos).cuda(), tp)
    tree = g.g4_build_tree(ctx, g.particles(x, y, z, torch.from_numpy(m).cuda()), tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    out = g.g4_tree_force(ctx, tree, g.walk_params(kernel=2, criterion=0, theta=1e-6, ewald=table))
    a = _stack(out)
    scale = (1.0 / 64) / 0.25 ** 2
    print("lattice |a| max", np.abs(a).max(), "pair scale", scale)
    assert np.abs(a).max() <= 1e-5 * scale


def test_kernel_2_needs_a_table_and_a_periodic_tree(g, ctx, table):
    tree, _, _, eps = _case(g, ctx, 300, 44)
    with pytest.raises(g.G4Error):
        g.g4_tree_force(ctx, tree, g.walk_params(kernel=2, eps0=eps))


def test_gpu_ewald_direct_sum_matches_the_oracle(g, ctx):
    """The FP64 direct sum with exact Ewald sums per pair (kernel 2 of
    g4_direct_force) against the oracle's, all targets and sampled targets."""
    ps = workloads.clustered_box(300, seed=45, nhalo=3)
    tp = g.tree_params(True, 1.0, leaf_max=8)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(ps.pos).cuda(), tp)
    m32 = ps.mass.astype(np.float32)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    wp = g.walk_params(kernel=2, eps0=0.003)
    out = g.g4_direct_force(ctx, p, tp, wp, want_pot=True)
    st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    ref, pot = oracle.direct(X, Y, Z, m32.astype(np.float64), 1.0 / 2 ** 32, kernel=2, eps0=0.003, nthreads=16)
    a = _stack(out)
    np.testing.assert_allclose(a, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(out["pot"].cpu().numpy(), pot, rtol=1e-9, atol=1e-11 * np.abs(pot).max())
    tg = np.array([0, 17, 299], dtype=np.int64)
    o2 = g.g4_direct_force(ctx, p, tp, wp, targets=torch.from_numpy(tg).cuda(), want_pot=False)
    np.testing.assert_allclose(_stack(o2), ref[tg], rtol=1e-9, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("det", [0, 1])
def test_periodic_fmm_parity_with_the_oracle(g, ctx, table, det):
    """The FMM with the Ewald correction (kernel 2), both summation modes,
    against the oracle's periodic FMM: the same interactions, forces and
    potentials at FP32 round-off, total momentum kept."""
    ps = workloads.clustered_box(4000, seed=46, nhalo=12)
    tp = g.tree_params(True, 1.0, leaf_max=16)
    x, y, z = g.g4_quantize(ctx, torch.from_numpy(ps.pos).cuda(), tp)
    m32 = ps.mass.astype(np.float32)
    p = g.particles(x, y, z, torch.from_numpy(m32).cuda())
    tree = g.g4_build_tree(ctx, p, tp)
    g.g4_compute_multipoles(ctx, tree, 3)
    st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    ot = oracle.Tree(X, Y, Z, m32.astype(np.float64), True, 1.0, 16)
    eps = (128 ** 3 / 4000) ** (1 / 3) / (40 * 128)
    out = g.g4_fmm_force(ctx, tree, g.fmm_params(kernel=2, theta=0.5, eps0=eps, deterministic=det, ewald=table),
                         want_pot=True, want_stats=True)
    acc, pot, stt = ot.fmm(kernel=2, theta=0.5, eps0=eps)
    _parity(_stack(out), acc, label=f"periodic fmm det={det}")
    assert np.median(np.abs(out["pot"].cpu().numpy() - pot) / np.abs(pot)) < 1e-5
    s = out["stats"]
    for k, v in zip(("n_pp", "n_pn", "n_nn"), stt):
        assert abs(s[k] - int(v)) <= 1e-3 * max(1, int(v)), (k, s[k], int(v))
    a = _stack(out)
    assert np.abs((m32[:, None].astype(np.float64) * a).sum(0)).max() <= 1e-6 * (m32[:, None] * np.abs(a)).sum()
