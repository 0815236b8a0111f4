"""Pins of the oracle's expansions at orders p = 4 and 5 (Appendix A,
"Multipole extensions at different order"): the printed Newtonian g_n, the
g_n recursion of the short-range kernel by finite differences, the full
derivative tensors D4 and D5 as successive gradients (trace-free for the
Newtonian kernel), and the convergence of the one-sided walk with p: each
order adds the next term of the expansion, so a compact cluster seen from far
away has a force error that falls by about l/r per order."""
import math

import numpy as np
import pytest

import oracle


def test_newtonian_gn_are_the_printed_values():
    r = 0.37
    g = oracle.gn_ext(0, r, 0.0, 7)
    printed = [1 / r, -1 / r ** 3, 3 / r ** 5, -15 / r ** 7, 105 / r ** 9, -945 / r ** 11, 10395 / r ** 13,
               -135135 / r ** 15]
    np.testing.assert_allclose(g, printed, rtol=1e-14)


@pytest.mark.parametrize("kernel,alpha", [(0, 0.0), (1, 3.0)])
def test_gn_recursion_by_finite_differences(kernel, alpha):
    """g_{n+1} = (1/r) d g_n / dr for n = 0..5."""
    for r in (0.05, 0.3, 0.9):
        h = 1e-5 * r
        g = oracle.gn_ext(kernel, r, alpha, 6)
        gp = oracle.gn_ext(kernel, r + h, alpha, 6)
        gm = oracle.gn_ext(kernel, r - h, alpha, 6)
        for n in range(6):
            fd = (gp[n] - gm[n]) / (2 * h) / r
            assert abs(fd - g[n + 1]) <= 1e-6 * abs(g[n + 1]) + 1e-9 * abs(g[n]) / r ** 2, (kernel, r, n)


@pytest.mark.parametrize("kernel,alpha", [(0, 0.0), (1, 2.0)])
def test_derivative_tensors_are_successive_gradients(kernel, alpha):
    rv = np.array([0.21, -0.13, 0.34])
    h = 1e-5
    for n in (3, 4):
        D = oracle.d_full(kernel, rv, n, alpha)
        Dn1 = oracle.d_full(kernel, rv, n + 1, alpha)
        for k in range(3):
            e = np.zeros(3); e[k] = h
            fd = (oracle.d_full(kernel, rv + e, n, alpha) - oracle.d_full(kernel, rv - e, n, alpha)) / (2 * h)
            np.testing.assert_allclose(Dn1[..., k], fd, rtol=1e-5, atol=1e-7 * np.abs(Dn1).max())
        # fully symmetric
        assert np.allclose(Dn1, np.swapaxes(Dn1, 0, n), rtol=1e-12, atol=0)
    if kernel == 0:
        # 1/r is harmonic: every trace of D4 and D5 vanishes
        D5 = oracle.d_full(0, rv, 5)
        assert np.abs(np.einsum("iijkl->jkl", D5)).max() < 1e-9 * np.abs(D5).max()
        D4 = oracle.d_full(0, rv, 4)
        assert np.abs(np.einsum("ijjk->ik", D4)).max() < 1e-9 * np.abs(D4).max()


def _cluster_case():
    """A lumpy cluster of 60 particles (radius ~0.02, off-centre clumps so
    that every multipole is present) and a target 0.25 away, in an isolated
    root; with leaf size 8 the cluster is split into a few nodes that the
    target accepts whole."""
    rng = np.random.default_rng(3)
    c = np.array([0.61, 0.43, 0.52])
    pts = c + 0.012 * rng.normal(size=(60, 3)) + np.where(rng.uniform(size=(60, 1)) < 0.3, 0.015, 0.0)
    tgt = np.array([[0.61 - 0.25, 0.43 + 0.02, 0.52 - 0.03]])
    pos = np.concatenate([tgt, pts])
    m = np.concatenate([[1e-6], rng.uniform(0.5, 1.5, 60)])
    st, X, Y, Z = oracle.quantize(pos, False, 1.0, (0.0, 0.0, 0.0))
    assert st == 0
    return X, Y, Z, m


def test_walk_error_falls_with_the_order():
    """The target's force from the cluster, accepted as one node: the error
    against the direct sum falls by a factor of several per order from p = 2
    to p = 5, so the octupole force term (p = 4) and the hexadecapole term
    (p = 5) each remove the leading error of the order below."""
    X, Y, Z, m = _cluster_case()
    ref, pref = oracle.direct(X, Y, Z, m, 2.0 ** -31, targets=np.array([0]))
    t = oracle.Tree(X, Y, Z, m, False, 1.0, 8)
    errs, perrs = [], []
    for p in (2, 3, 4, 5):
        acc, pot, cnt = t.walk(kernel=0, criterion=0, theta=0.5, order=p, targets=np.array([0]))
        assert cnt[0, 1] >= 1 and cnt[0, 0] <= 4
        errs.append(np.linalg.norm(acc[0] - ref[0]) / np.linalg.norm(ref[0]))
        perrs.append(abs(pot[0] - pref[0]) / abs(pref[0]))
    print("force errors by p:", errs, "potential errors:", perrs)
    for k in range(3):
        assert errs[k + 1] < errs[k] / 3, errs
    # the potential gains the Q3 term at p = 3 and the Q4 term at p = 4
    assert perrs[1] < perrs[0] / 3 and perrs[2] < perrs[1] / 3


def test_higher_orders_converge_to_direct_sum_and_follow_alpha():
    """theta -> 0 at p = 4, 5 is the direct sum; the relative criterion at
    p = 5 with alpha = 1e-3 keeps the 90th percentile of the errors near alpha."""
    rng = np.random.default_rng(8)
    n = 800
    pos = np.concatenate([rng.uniform(0.2, 0.8, size=(n // 2, 3)), 0.5 + 0.03 * rng.normal(size=(n // 2, 3))])
    m = rng.uniform(0.5, 1.5, n) / n
    st, X, Y, Z = oracle.quantize(pos, False, 1.0, (0.0, 0.0, 0.0))
    ref, _ = oracle.direct(X, Y, Z, m, 2.0 ** -31, eps0=1e-3, nthreads=8)
    t = oracle.Tree(X, Y, Z, m, False, 1.0, 8)
    for p in (4, 5):
        acc, _, _ = t.walk(kernel=0, criterion=0, theta=1e-9, order=p, eps0=1e-3, nthreads=8)
        np.testing.assert_allclose(acc, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    aseed = np.linalg.norm(ref, axis=1)
    acc, _, cnt = t.walk(kernel=0, criterion=1, alpha=1e-3, order=5, eps0=1e-3, aseed=aseed, nthreads=8)
    err = np.linalg.norm(acc - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert cnt[:, 1].sum() > 0
    assert 1e-3 / 30 < np.percentile(err, 90) < 3e-3
