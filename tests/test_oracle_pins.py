"""Pins of the FP64 oracle against what the paper and mathematics fix.

Every test here runs on the CPU and checks the oracle against something other
than itself: values printed in the paper, closed forms, finite-difference
derivatives, numerical integration of the printed spline kernel, invariants,
and brute force on tiny inputs.  A dropped term, a wrong sign or a transposed
index in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import workloads

H = 0.028  # softening edge h = 2.8 eps0 for eps0 = 0.01


# ---------------------------------------------------------------- integers
def test_integer_wrap_worked_example():
    """Sec. "Integer coordinates": with one byte, 200 - 30 read as signed is -86,
    and 200 + 100 wraps to 44.  The same holds in the top byte of 32-bit ints."""
    a, b = np.uint8(200), np.uint8(30)
    assert int(np.array(a - b, dtype=np.uint8).view(np.int8)) == -86
    assert int(np.uint8((int(a) + 100) % 256)) == 44
    L = 1.0
    pos = np.array([[200 / 256, 0.5, 0.5], [30 / 256, 0.5, 0.5], [300 / 256, 0.5, 0.5]])
    st, X, Y, Z = oracle.quantize(pos, True, L)
    assert st == 0
    assert X[0] == 200 << 24 and X[1] == 30 << 24 and X[2] == 44 << 24
    assert int(np.array([X[0] - X[1]], dtype=np.uint32).view(np.int32)[0]) == -86 << 24


def test_isolated_root_mapping():
    """Sec. "Non-periodic potentials": the root maps into a sub-range of the
    integer space so that differences never wrap; leaving it is reported."""
    pos = np.array([[0.0, 0.0, 0.0], [1.0 - 1e-12, 0.5, 0.25]])
    st, X, Y, Z = oracle.quantize(pos, False, 1.0, (0.0, 0.0, 0.0))
    assert st == 0
    assert X[0] == 2 ** 30 and Y[1] == 2 ** 30 + 2 ** 30 and Z[1] == 2 ** 30 + 2 ** 29
    assert X[1] < 3 * 2 ** 30
    st, *_ = oracle.quantize(np.array([[1.5, 0.0, 0.0]]), False, 1.0, (0.0, 0.0, 0.0))
    assert st == -5


# ---------------------------------------------------------------- softening
def w_m4(q):
    """Cubic spline kernel as printed in the paper's SPH kernel section."""
    if q <= 0.5:
        return 8 / math.pi * (1 - 6 * q * q + 6 * q ** 3)
    if q <= 1.0:
        return 8 / math.pi * 2 * (1 - q) ** 3
    return 0.0


def test_softening_depth_and_edge():
    """phi(0) = -G m / eps0, and the force is Newtonian for r >= 2.8 eps0."""
    eps0 = 0.01
    assert oracle.soft_W(0.0, 2.8 * eps0) == pytest.approx(1 / eps0, rel=1e-14)
    for r in [H, 1.5 * H, 10 * H]:
        assert oracle.soft_K(r, H) == pytest.approx(r ** -3, rel=1e-14)
        assert oracle.soft_W(r, H) == pytest.approx(1 / r, rel=1e-14)


def test_softening_enclosed_mass_of_printed_kernel():
    """K(r) r^3 equals the mass of the spline density (8/(pi h^3)) w(r/h) inside r."""
    for u in [0.05, 0.2, 0.49, 0.5, 0.51, 0.7, 0.95, 1.0]:
        m_in, _ = integrate.quad(lambda q: 4 * math.pi * q * q * w_m4(q), 0.0, u, epsabs=1e-14, epsrel=1e-13)
        r = u * H
        assert oracle.soft_K(r, H) * r ** 3 == pytest.approx(m_in, rel=1e-10, abs=1e-14)


def test_softening_force_is_gradient_of_potential():
    for u in [0.1, 0.3, 0.45, 0.55, 0.8, 0.99, 1.3]:
        r, d = u * H, 1e-6 * H
        dW = (oracle.soft_W(r + d, H) - oracle.soft_W(r - d, H)) / (2 * d)
        assert oracle.soft_K(r, H) == pytest.approx(-dW / r, rel=1e-7)


def test_softening_continuity():
    for u in [0.5, 1.0]:
        lo, hi = (u - 1e-12) * H, (u + 1e-12) * H
        assert oracle.soft_K(lo, H) == pytest.approx(oracle.soft_K(hi, H), rel=1e-9)
        assert oracle.soft_W(lo, H) == pytest.approx(oracle.soft_W(hi, H), rel=1e-9)


# ---------------------------------------------------------------- short range
RS = 1.25 / 256
ALPHA = 0.5 / RS  # r_s = 1/(2 alpha)
EPS_SR = 1.0 / (40 * 128)
H_SR = 2.8 * EPS_SR


def test_short_range_potential_is_eqnpo4():
    """Per source, eq. (eqnpo4) gives -[W_soft(r) - erf(alpha r)/r] up to a constant."""
    for r in [1e-6, 0.2 * H_SR, 0.7 * H_SR, H_SR, 2 * RS, 4.5 * RS]:
        ref = oracle.soft_W(r, H_SR) - special.erf(ALPHA * r) / r
        assert oracle.sr_W(r, H_SR, ALPHA) == pytest.approx(ref, rel=1e-12)


def test_short_range_force_is_gradient_of_potential():
    for r in [0.3 * H_SR, 0.6 * H_SR, 1.5 * H_SR, RS, 3 * RS, 6 * RS]:
        d = 1e-6 * r
        dW = (oracle.sr_W(r + d, H_SR, ALPHA) - oracle.sr_W(r - d, H_SR, ALPHA)) / (2 * d)
        assert oracle.sr_K(r, H_SR, ALPHA) == pytest.approx(-dW / r, rel=1e-6)


def test_short_range_suppression_at_cutoff():
    """Sec. "TreePM approach": at R_cut = 7 the force and potential are suppressed
    to around 1e-5 of Newtonian; R_cut = 4.5 only reaches ~1e-2."""
    f7 = oracle.sr_K(7 * RS, 0.0, ALPHA) * (7 * RS) ** 3
    p7 = oracle.sr_W(7 * RS, 0.0, ALPHA) * (7 * RS)
    f45 = oracle.sr_K(4.5 * RS, 0.0, ALPHA) * (4.5 * RS) ** 3
    assert 5e-6 < f7 < 5e-5 and p7 < 1e-5
    assert 5e-3 < f45 < 5e-2


def test_short_range_newtonian_limit():
    for r in [0.5 * H, 2 * H]:
        assert oracle.sr_K(r, H, 1e-9) == pytest.approx(oracle.soft_K(r, H), rel=1e-12)


# ---------------------------------------------------------------- g_n and D_n
def test_gn_newtonian_appendix_values():
    """Appendix A: g0 = 1/r, g1 = -1/r^3, g2 = 3/r^5, g3 = -15/r^7."""
    for r in [0.3, 1.0, 7.0]:
        g = oracle.gn(0, r)
        np.testing.assert_allclose(g, [1 / r, -1 / r ** 3, 3 / r ** 5, -15 / r ** 7], rtol=1e-14)


def _g_sr(r):
    return special.erfc(ALPHA * r) / r


def _deriv(f, r, k, h):
    """k-th derivative by a 9-point central stencil applied recursively."""
    if k == 0:
        return f(r)
    c = [1 / 280, -4 / 105, 1 / 5, -4 / 5, 0, 4 / 5, -1 / 5, 4 / 105, -1 / 280]
    return sum(ci * _deriv(f, r + (i - 4) * h, k - 1, h) for i, ci in enumerate(c)) / h


def test_gn_short_range_appendix_forms():
    """Appendix A: g1 = g'/r, g2 = (g'' - g'/r)/r^2, g3 = (g''' - 3 g''/r + 3 g'/r^2)/r^3."""
    for r in [0.5 * RS, RS, 3 * RS]:
        h = 0.02 * r
        d1, d2, d3 = (_deriv(_g_sr, r, k, h) for k in (1, 2, 3))
        g = oracle.gn(1, r, ALPHA)
        assert g[0] == pytest.approx(_g_sr(r), rel=1e-13)
        assert g[1] == pytest.approx(d1 / r, rel=1e-9)
        assert g[2] == pytest.approx((d2 - d1 / r) / r ** 2, rel=1e-7)
        assert g[3] == pytest.approx((d3 - 3 * d2 / r + 3 * d1 / r ** 2) / r ** 3, rel=1e-5)


def test_gn_short_range_newtonian_limit():
    g = oracle.gn(1, 0.7, 1e-14)
    np.testing.assert_allclose(g, oracle.gn(0, 0.7), rtol=1e-12)


@pytest.mark.parametrize("kernel", [0, 1])
def test_Dn_are_successive_gradients(kernel):
    """D_n = grad^n g (eqs. eqngderiv0-eqngderiv), checked by central differences."""
    alpha = ALPHA if kernel else 0.0
    rv = np.array([0.6, -0.35, 0.8]) * (RS if kernel else 1.0)
    h = 1e-5 * np.linalg.norm(rv)
    D = oracle.Dn(kernel, rv, alpha)
    for n in range(3):
        num = []
        for k in range(3):
            e = np.zeros(3); e[k] = h
            num.append((np.asarray(oracle.Dn(kernel, rv + e, alpha)[n]) - np.asarray(oracle.Dn(kernel, rv - e, alpha)[n])) / (2 * h))
        num = np.moveaxis(np.array(num), 0, -1)
        np.testing.assert_allclose(D[n + 1], num, rtol=2e-6, atol=2e-6 * np.abs(D[n + 1]).max())


def test_Dn_newtonian_trace_free():
    _, D1, D2, D3 = oracle.Dn(0, np.array([0.3, 0.4, -1.2]))
    assert abs(np.trace(D2)) < 1e-13 * np.abs(D2).max()
    assert np.abs(np.einsum("iik->k", D3)).max() < 1e-13 * np.abs(D3).max()
    np.testing.assert_allclose(D3, np.transpose(D3, (1, 0, 2)), rtol=1e-15)
    np.testing.assert_allclose(D3, np.transpose(D3, (2, 1, 0)), rtol=1e-15)


# ---------------------------------------------------------------- tree
def _node_set_by_definition(X, Y, Z, periodic, B, maxd=21):
    """Node (l, cell) exists iff l == 0 or its parent cell holds > B particles."""
    S = 32 if periodic else 31
    corner = 0 if periodic else 2 ** 30
    rel = [(np.asarray(A, np.uint64) - corner) & 0xFFFFFFFF for A in (X, Y, Z)]
    out = set()
    parent_big = None
    for lev in range(0, maxd + 1):
        sh = np.uint64(S - lev)
        cells = np.stack([r >> sh for r in rel], axis=1)
        keys, counts = np.unique(cells, axis=0, return_counts=True)
        for c, k in zip(keys, counts):
            if lev == 0 or (tuple(int(v) >> 1 for v in c) in parent_big):
                out.add((lev, int(c[0]), int(c[1]), int(c[2]), int(k)))
        parent_big = {tuple(int(v) for v in c) for c, k in zip(keys, counts)
                      if k > B and (lev == 0 or (lev, int(c[0]), int(c[1]), int(c[2]), int(k)) in out)}
    return out


@pytest.mark.parametrize("periodic", [False, True])
def test_tree_node_set_matches_definition(periodic):
    """Sec. "Geometry of the tree": a node is split only when it holds more than B particles."""
    if periodic:
        ps = workloads.clustered_box(3000, seed=5, nhalo=20)
        st, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    else:
        ps = workloads.plummer(3000, seed=4)
        org, side = workloads.isolated_root(ps.pos)
        st, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    assert st == 0
    B = 8
    t = oracle.Tree(X, Y, Z, ps.mass, periodic, 1.0, B)
    level, cell, count, leaf = t.nodes()
    got = {(int(l), int(c[0]), int(c[1]), int(c[2]), int(k)) for l, c, k in zip(level, cell, count)}
    assert got == _node_set_by_definition(X, Y, Z, periodic, B)
    assert np.all((count <= B) | (leaf == 0) | (level == 21))
    assert np.all(count[leaf == 0] > B)
    assert count[leaf == 1].sum() == len(X)


def test_tree_coincident_particles_depth_cap():
    X = np.full(20, 123456789, np.uint32)
    t = oracle.Tree(X, X, X, np.ones(20), True, 1.0, 8)
    level, cell, count, leaf = t.nodes()
    assert level.max() == 21 and count[level == 21][0] == 20 and leaf[level == 21][0] == 1


def test_moments_parallel_axis_consistency():
    """Each node's moments equal the sum of its constituents' moments shifted to its
    centre of mass (parallel-axis theorem), the relation an upward pass uses."""
    ps = workloads.plummer(2000, seed=7)
    org, side = workloads.isolated_root(ps.pos)
    _, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    t = oracle.Tree(X, Y, Z, ps.mass, False, side, 8)
    t.compute_moments()
    mass, com, q2p, q3p = t.moments()
    level, cell, count, leaf = t.nodes()

    def full2(q):
        xx, xy, xz, yy, yz, zz = q
        return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])

    def full3(q):
        idx = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2), (2, 2, 2)]
        T = np.zeros((3, 3, 3))
        import itertools
        for v, (i, j, k) in zip(q, idx):
            for p in set(itertools.permutations((i, j, k))):
                T[p] = v
        return T

    # particle positions relative to the root corner
    pos = np.stack([(X.astype(np.float64) - 2 ** 30), (Y.astype(np.float64) - 2 ** 30),
                    (Z.astype(np.float64) - 2 ** 30)], axis=1) * (side / 2 ** 31)
    # children of each node: nodes at level+1 with cell>>1 == cell
    bylev = {}
    for q in range(len(level)):
        bylev.setdefault(int(level[q]), []).append(q)
    cellkey = {(int(level[q]), *map(int, cell[q])): q for q in range(len(level))}
    checked = 0
    for q in range(len(level)):
        if leaf[q]:
            lo = cell[q].astype(np.int64) << (31 - level[q])
            inside = np.all((np.stack([X, Y, Z], 1).astype(np.int64) - 2 ** 30 >> (31 - level[q])) == cell[q], axis=1)
            ms, ss, Q2s, Q3s = ps.mass[inside], pos[inside], [np.zeros((3, 3))] * inside.sum(), [np.zeros((3, 3, 3))] * inside.sum()
        else:
            ch = [cellkey[k] for k in [(int(level[q]) + 1, 2 * int(cell[q][0]) + a, 2 * int(cell[q][1]) + b, 2 * int(cell[q][2]) + c)
                                       for a in (0, 1) for b in (0, 1) for c in (0, 1)] if k in cellkey]
            ms, ss = mass[ch], com[ch]
            Q2s, Q3s = [full2(q2p[c]) for c in ch], [full3(q3p[c]) for c in ch]
        M = ms.sum()
        s = (ms[:, None] * ss).sum(0) / M
        Q2 = sum(Q2c + mc * np.outer(sc - s, sc - s) for mc, sc, Q2c in zip(ms, ss, Q2s))
        Q3 = 0
        for mc, sc, Q2c, Q3c in zip(ms, ss, Q2s, Q3s):
            d = sc - s
            Q3 = Q3 + Q3c + np.einsum("i,jk->ijk", d, Q2c) + np.einsum("j,ik->ijk", d, Q2c) \
                + np.einsum("k,ij->ijk", d, Q2c) + mc * np.einsum("i,j,k->ijk", d, d, d)
        assert mass[q] == pytest.approx(M, rel=1e-13)
        np.testing.assert_allclose(com[q], s, rtol=0, atol=1e-12 * side)
        scale2 = M * (side / 2 ** level[q]) ** 2
        np.testing.assert_allclose(full2(q2p[q]), Q2, rtol=0, atol=1e-11 * scale2)
        np.testing.assert_allclose(full3(q3p[q]), Q3, rtol=0, atol=1e-11 * scale2 * side / 2 ** level[q])
        checked += 1
    assert checked == len(level)


# ---------------------------------------------------------------- direct sums
def test_direct_two_body_and_third_law():
    st, X, Y, Z = oracle.quantize(np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]]), False, 1.0, (0, 0, 0))
    m = np.array([2.0, 3.0])
    acc, pot = oracle.direct(X, Y, Z, m, 1.0 / 2 ** 31, G=1.0, eps0=0.0)
    assert acc[0, 0] == pytest.approx(3.0 / 0.25, rel=1e-14) and acc[1, 0] == pytest.approx(-2.0 / 0.25, rel=1e-14)
    assert pot[0] == pytest.approx(-3.0 / 0.5, rel=1e-14)
    ps = workloads.plummer(64, seed=3)
    org, side = workloads.isolated_root(ps.pos)
    _, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    acc, _ = oracle.direct(X, Y, Z, ps.mass, side / 2 ** 31, G=1.0, eps0=0.01)
    net = (ps.mass[:, None] * acc).sum(0)
    assert np.abs(net).max() < 1e-14 * np.abs(ps.mass[:, None] * acc).sum()


def test_direct_long_double_brute_force():
    ps = workloads.plummer(48, seed=9)
    org, side = workloads.isolated_root(ps.pos)
    _, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    unit = side / 2 ** 31
    P = np.stack([X, Y, Z], 1).astype(np.longdouble) * np.longdouble(unit)
    ref = np.zeros((48, 3), np.longdouble)
    for i in range(48):
        for j in range(48):
            if i != j:
                d = P[j] - P[i]
                ref[i] += np.longdouble(ps.mass[j]) * d / np.sqrt((d * d).sum()) ** 3
    acc, _ = oracle.direct(X, Y, Z, ps.mass, unit, G=1.0, eps0=0.0)
    np.testing.assert_allclose(acc, ref.astype(np.float64), rtol=1e-12)


def test_periodic_nearest_image_and_translation_invariance():
    """Sec. "Integer coordinates" and the random-translation passage: the periodic
    direct sum is bitwise invariant under a common integer shift."""
    ps = workloads.clustered_box(400, seed=11, nhalo=5)
    _, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    kw = dict(kernel=1, G=1.0, eps0=EPS_SR, r_s=0.05, r_cut=np.inf)
    a0, p0 = oracle.direct(X, Y, Z, ps.mass, 2.0 ** -32, **kw)
    sh = np.uint32(2_987_654_321)
    a1, p1 = oracle.direct(X + sh, Y + np.uint32(17), Z - np.uint32(99), ps.mass, 2.0 ** -32, **kw)
    assert np.array_equal(a0, a1) and np.array_equal(p0, p1)
    # a pair 0.9 L apart along x interacts through the image 0.1 L away
    st, X, Y, Z = oracle.quantize(np.array([[0.05, 0.5, 0.5], [0.95, 0.5, 0.5]]), True, 1.0)
    acc, _ = oracle.direct(X, Y, Z, np.ones(2), 2.0 ** -32, kernel=1, G=1.0, eps0=0.0, r_s=1.0, r_cut=np.inf)
    assert acc[0, 0] < 0 and acc[0, 0] == pytest.approx(-oracle.sr_K(0.1, 0.0, 0.5) * 0.1, rel=1e-7)


# ---------------------------------------------------------------- walks
def _plummer_tree(n=2000, seed=21, B=8):
    ps = workloads.plummer(n, seed=seed)
    org, side = workloads.isolated_root(ps.pos)
    _, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    t = oracle.Tree(X, Y, Z, ps.mass, False, side, B)
    t.compute_moments()
    return ps, t, side


def test_walk_theta_to_zero_is_direct_sum():
    ps, t, side = _plummer_tree()
    acc, pot, cnt = t.walk(kernel=0, criterion=0, theta=1e-9, eps0=0.01)
    ref, pref = oracle.direct(t.X, t.Y, t.Z, t.mass, t.unit, G=1.0, eps0=0.01)
    np.testing.assert_allclose(acc, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
    np.testing.assert_allclose(pot, pref, rtol=1e-12)
    assert np.all(cnt[:, 1] == 0) and np.all(cnt[:, 0] == t.n - 1)


def test_relative_walk_alpha_to_zero_is_direct_sum():
    ps, t, side = _plummer_tree(800)
    seed = np.ones(t.n)
    acc, _, _ = t.walk(kernel=0, criterion=1, alpha=1e-30, aseed=seed, eps0=0.01)
    ref, _ = oracle.direct(t.X, t.Y, t.Z, t.mass, t.unit, G=1.0, eps0=0.01)
    np.testing.assert_allclose(acc, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_treepm_walk_theta_to_zero_is_direct_sum():
    ps = workloads.clustered_box(1500, seed=13, nhalo=10)
    _, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    t = oracle.Tree(X, Y, Z, ps.mass, True, 1.0, 8)
    kw = dict(kernel=1, G=1.0, eps0=EPS_SR, r_s=0.02, r_cut=np.inf)
    acc, pot, _ = t.walk(criterion=0, theta=1e-9, **kw)
    ref, pref = oracle.direct(X, Y, Z, ps.mass, 2.0 ** -32, **kw)
    np.testing.assert_allclose(acc, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(pot, pref, rtol=1e-10)


def test_treepm_cutoff_drops_only_far_nodes():
    """With r_cut, a theta -> 0 walk keeps every pair closer than r_cut and only
    pairs beyond it can be missing (nodes dropped by their nearest edge)."""
    ps = workloads.clustered_box(1500, seed=14, nhalo=10)
    _, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    t = oracle.Tree(X, Y, Z, ps.mass, True, 1.0, 8)
    rs, rc = 0.02, 0.09
    acc, _, cnt = t.walk(criterion=0, theta=1e-9, kernel=1, eps0=EPS_SR, r_s=rs, r_cut=rc)
    near, _ = oracle.direct(X, Y, Z, ps.mass, 2.0 ** -32, kernel=1, eps0=EPS_SR, r_s=rs, r_cut=rc, truncate=True)
    full, _ = oracle.direct(X, Y, Z, ps.mass, 2.0 ** -32, kernel=1, eps0=EPS_SR, r_s=rs, r_cut=np.inf)
    # every pair within r_cut is present: the walk lies between the two sums
    # in the sense that walk - near is made of pairs beyond r_cut only
    far_max = oracle.sr_K(rc, 0.0, 0.5 / rs) * rc * ps.mass[0]
    d = np.linalg.norm(acc - near, axis=1)
    assert np.all(d <= far_max * (t.n - 1) + 1e-12)
    pairs_in = np.array([np.sum(np.linalg.norm(((np.stack([X, Y, Z], 1).astype(np.int64) - np.array([X[i], Y[i], Z[i]], np.int64) + 2 ** 31) % 2 ** 32 - 2 ** 31) * 2.0 ** -32, axis=1) <= rc) - 1 for i in range(0, t.n, 50)])
    assert np.all(cnt[::50, 0] >= pairs_in)
    assert np.all(cnt[:, 0] < t.n - 1)  # something was dropped
    assert np.abs(full - acc).max() > 0


def _pair_errors(theta_A, theta_B, rng, ngrp=10):
    """Two cubes of 10 random equal-mass particles, COMs a unit distance apart."""
    lA, lB = theta_A, theta_B
    pa = rng.uniform(-0.5, 0.5, (ngrp, 3)) * lA
    pb = rng.uniform(-0.5, 0.5, (ngrp, 3)) * lB
    pa -= pa.mean(0)
    pb -= pb.mean(0)
    e = rng.normal(size=3); e /= np.linalg.norm(e)
    pb += e
    m = np.full(ngrp, 1.0)
    aAf, aBf, aAt, aBt = oracle.two_groups(pa, m, pb, m)
    # exact forces of B on A and A on B
    refA = np.array([sum(m[j] * (pb[j] - pa[i]) / np.linalg.norm(pb[j] - pa[i]) ** 3 for j in range(ngrp)) for i in range(ngrp)])
    refB = np.array([sum(m[j] * (pa[j] - pb[i]) / np.linalg.norm(pa[j] - pb[i]) ** 3 for j in range(ngrp)) for i in range(ngrp)])
    err = lambda a, r: np.mean(np.linalg.norm(a - r, axis=1) / np.linalg.norm(r, axis=1))
    return err(aAf, refA), err(aBf, refB), err(aAt, refA), err(aBt, refB), (m[:, None] * (aAf)).sum(0) + (m[:, None] * aBf).sum(0)


def test_two_node_fmm_asymptote_and_tree_ratio():
    """Sec. "The FMM force accuracy between two interacting nodes" (p = 3):
    node A's error tends to ~0.009 for theta_A -> 0 at theta_B = 0.5, and FMM's
    error is ~4x the tree's at the same opening angle (loose pins)."""
    rng = np.random.default_rng(1859)
    asym = np.median([_pair_errors(1e-4, 0.5, rng)[0] for _ in range(300)])
    assert 0.009 / 1.6 < asym < 0.009 * 1.6
    ratios = []
    for th in (0.2, 0.3, 0.5):
        e = [_pair_errors(th, th, rng) for _ in range(300)]
        fmm = np.median([x[0] for x in e] + [x[1] for x in e])
        tree = np.median([x[2] for x in e] + [x[3] for x in e])
        ratios.append(fmm / tree)
    assert 2.5 < np.median(ratios) < 6.5


def test_two_node_momentum_and_tree_order():
    """FMM pair forces cancel exactly (manifest momentum conservation); the tree
    force error falls as theta^3 at p = 3 (force to second order)."""
    rng = np.random.default_rng(2045)
    for _ in range(20):
        *_, net = _pair_errors(0.4, 0.3, rng)
        assert np.abs(net).max() < 1e-13
    e1 = np.median([_pair_errors(1e-4, 0.4, rng)[2] for _ in range(400)])
    e2 = np.median([_pair_errors(1e-4, 0.2, rng)[2] for _ in range(400)])
    assert 5.0 < e1 / e2 < 12.0


def test_plummer_closed_form_acceleration():
    """Binned radial acceleration of the N = 8192 Plummer sphere against
    -G M(<r)/r^2 with M(<r) = r^3/(1+r^2)^{3/2} / M(<20)."""
    ps = workloads.plummer(8192, seed=1)
    org, side = workloads.isolated_root(ps.pos)
    _, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    t = oracle.Tree(X, Y, Z, ps.mass, False, side, 8)
    a0, _, _ = t.walk(criterion=0, theta=0.7, eps0=0.01, nthreads=8)
    acc, _, _ = t.walk(criterion=1, alpha=0.005, aseed=np.linalg.norm(a0, axis=1), eps0=0.01, nthreads=8)
    r = np.linalg.norm(ps.pos, axis=1)
    ar = (acc * ps.pos).sum(1) / r
    edges = np.array([0.3, 0.5, 0.8, 1.2, 2.0, 3.5])
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        rr = r[sel]
        model = -(rr ** 3 / (1 + rr ** 2) ** 1.5 / workloads.PLUMMER_MASS_FRACTION_R20) / rr ** 2
        assert np.mean(ar[sel]) == pytest.approx(np.mean(model), rel=0.05)


def test_relative_criterion_error_tracks_alpha():
    """Sec. "Force errors for an isolated particle distribution": alpha roughly
    equals the 90th-percentile force error (loose), and errors fall with alpha."""
    ps, t, side = _plummer_tree(4000, seed=31)
    ref, _ = oracle.direct(t.X, t.Y, t.Z, t.mass, t.unit, G=1.0, eps0=0.01, nthreads=8)
    a0, _, _ = t.walk(criterion=0, theta=0.7, eps0=0.01, nthreads=8)
    seed = np.linalg.norm(a0, axis=1)
    p90 = []
    for alpha in (0.02, 0.005, 0.00125):
        acc, _, _ = t.walk(criterion=1, alpha=alpha, aseed=seed, eps0=0.01, nthreads=8)
        p90.append(np.percentile(workloads.relative_errors(acc, ref), 90))
        assert alpha / 30 < p90[-1] < alpha * 3
    assert p90[0] > p90[1] > p90[2]


# ---------------------------------------------------------------- FMM
def test_fmm_theta_to_zero_is_direct_sum():
    ps, t, side = _plummer_tree(600, seed=41, B=16)
    acc, pot, st = t.fmm(kernel=0, theta=1e-9, eps0=0.01)
    ref, pref = oracle.direct(t.X, t.Y, t.Z, t.mass, t.unit, G=1.0, eps0=0.01)
    np.testing.assert_allclose(acc, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
    np.testing.assert_allclose(pot, pref, rtol=1e-12)
    assert st[1] == 0 and st[2] == 0 and st[0] == 600 * 599 // 2


@pytest.mark.parametrize("kernel", [0, 1])
def test_fmm_momentum_conservation(kernel):
    """Sec. "Fast multipole method": the symmetric expansion conserves momentum to
    machine precision; the errors against direct summation stay small."""
    if kernel == 0:
        ps, t, side = _plummer_tree(3000, seed=43, B=16)
        kw = dict(kernel=0, eps0=0.01, theta=0.5)
        ref, _ = oracle.direct(t.X, t.Y, t.Z, t.mass, t.unit, G=1.0, eps0=0.01, nthreads=8)
    else:
        ps = workloads.clustered_box(3000, seed=44, nhalo=20)
        _, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
        t = oracle.Tree(X, Y, Z, ps.mass, True, 1.0, 16)
        kw = dict(kernel=1, eps0=EPS_SR, r_s=0.03, r_cut=0.135, theta=0.5)
        ref, _ = oracle.direct(X, Y, Z, ps.mass, 2.0 ** -32, kernel=1, eps0=EPS_SR, r_s=0.03, r_cut=np.inf, nthreads=8)
    acc, pot, st = t.fmm(**kw)
    net = (t.mass[:, None] * acc).sum(0)
    assert np.abs(net).max() < 1e-13 * (t.mass[:, None] * np.abs(acc)).sum()
    assert st[1] > 0 and st[2] > 0
    err = workloads.relative_errors(acc, ref)
    assert np.percentile(err, 50) < 2e-2


def test_fmm_relative_criterion_limits_and_accuracy():
    """Relative node-node criterion (Sec. "Fast multipole method"): alpha -> 0
    opens every pair down to particles (the direct sum); at finite alpha the
    interactions stay symmetric (momentum to round-off) and the errors shrink
    as alpha does, with the 90th percentile following alpha within a factor
    of a few (the criterion bounds the error of each interaction relative to
    the target's |a|)."""
    ps, t, side = _plummer_tree(1500, seed=45, B=16)
    ref, _ = oracle.direct(t.X, t.Y, t.Z, t.mass, t.unit, G=1.0, eps0=0.01, nthreads=8)
    aseed = np.linalg.norm(ref, axis=1)
    acc, _, st = t.fmm(kernel=0, eps0=0.01, criterion=1, alpha=1e-14, aseed=aseed)
    np.testing.assert_allclose(acc, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert st[1] == 0 and st[2] == 0
    p90 = []
    for alpha in (0.01, 0.001):
        acc, _, st = t.fmm(kernel=0, eps0=0.01, criterion=1, alpha=alpha, aseed=aseed)
        net = (t.mass[:, None] * acc).sum(0)
        assert np.abs(net).max() < 1e-13 * (t.mass[:, None] * np.abs(acc)).sum()
        assert st[2] > 0
        err = workloads.relative_errors(acc, ref)
        p90.append(np.percentile(err, 90))
        assert alpha / 30 < p90[-1] < alpha * 3, (alpha, p90[-1])
    assert p90[1] < p90[0] / 3


def test_tree_is_not_momentum_conserving():
    """The one-sided tree does not conserve momentum (the contrast the paper draws)."""
    ps, t, side = _plummer_tree(3000, seed=43, B=16)
    acc, _, _ = t.walk(criterion=0, theta=0.7, eps0=0.01, nthreads=8)
    net = (t.mass[:, None] * acc).sum(0)
    assert np.abs(net).max() > 1e-9 * (t.mass[:, None] * np.abs(acc)).sum()


# ---------------------------------------------------------------- MLP
@pytest.mark.parametrize("tau", [0.0, 0.3])
def test_mlp_gradient_finite_differences(tau):
    rng = np.random.default_rng(5)
    w = rng.normal(scale=0.3, size=oracle.NPARAM)
    feat = rng.normal(size=(7, 8))
    target = rng.normal(size=7)
    loss, g = oracle.mlp_loss_grad(w, feat, target, tau)
    y = oracle.mlp_forward(w, feat)
    u = target - y
    ref = np.mean((y - target) ** 2) if tau == 0 else np.mean(np.where(u >= 0, tau * u, (tau - 1) * u))
    assert loss == pytest.approx(ref, rel=1e-13)
    for i in list(range(0, 512, 37)) + list(range(512, 4801, 211)) + [4800, 4736, 4672]:
        e = np.zeros(oracle.NPARAM); e[i] = 1e-6
        lp, _ = oracle.mlp_loss_grad(w + e, feat, target, tau)
        lm, _ = oracle.mlp_loss_grad(w - e, feat, target, tau)
        assert g[i] == pytest.approx((lp - lm) / 2e-6, rel=1e-5, abs=1e-9)


def test_mlp_silu_forward_special_case():
    """With zero hidden weights every unit is SiLU(b); SiLU(z) = z sigmoid(z)."""
    w = np.zeros(oracle.NPARAM)
    w[512:576] = 1.0          # b1 -> h1 = silu(1)
    w[4672:4736] = -2.0       # b2 -> h2 = silu(-2), W2 = 0
    w[4736:4800] = 0.5        # w3
    w[4800] = 0.25
    y = oracle.mlp_forward(w, np.ones((3, 8)))
    silu = lambda z: z / (1 + math.exp(-z))
    assert y == pytest.approx(np.full(3, 0.25 + 64 * 0.5 * silu(-2.0)), rel=1e-14)


def test_adam_first_step_is_signed_lr():
    """Adam's bias correction makes the first update -lr * g / (|g| + eps)."""
    w = np.zeros(5); m = np.zeros(5); v = np.zeros(5)
    g = np.array([3.0, -0.5, 1e-3, -7.0, 2.0])
    oracle.adam(w, g, m, v, lr=0.01, step=1, eps=0.0)
    np.testing.assert_allclose(w, -0.01 * np.sign(g), rtol=1e-12)


def test_threaded_build_and_moments_equal_serial():
    """The threaded tree build and moment sums (used to time the oracle on many
    cores) give the serial code's node set and, node by node, its moments."""
    ps = workloads.clustered_box(20000, seed=77, nhalo=40)
    _, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    t1 = oracle.Tree(X, Y, Z, ps.mass, True, 1.0, 8)
    t1.compute_moments()
    t4 = oracle.Tree(X, Y, Z, ps.mass, True, 1.0, 8, nthreads=4)
    t4.compute_moments(nthreads=4)
    k1 = {(int(l), *map(int, c), int(k)): i for i, (l, c, k) in enumerate(zip(*t1.nodes()[:3]))}
    k4 = {(int(l), *map(int, c), int(k)): i for i, (l, c, k) in enumerate(zip(*t4.nodes()[:3]))}
    assert k1.keys() == k4.keys()
    m1, m4 = t1.moments(), t4.moments()
    i1 = np.array([k1[k] for k in k1]); i4 = np.array([k4[k] for k in k1])
    for a, b in zip(m1, m4):
        np.testing.assert_allclose(a[i1], b[i4], rtol=1e-12, atol=1e-300)
    a1, _, c1 = t1.walk(criterion=0, theta=0.6, eps0=1e-4, targets=np.arange(0, 20000, 97))
    a4, _, c4 = t4.walk(criterion=0, theta=0.6, eps0=1e-4, targets=np.arange(0, 20000, 97), nthreads=4)
    np.testing.assert_allclose(a1, a4, rtol=1e-12)
    assert np.array_equal(c1, c4)
