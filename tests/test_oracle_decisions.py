"""Constructed cases that pin the oracle's decision rules one at a time.

The statistical pins (theta -> 0 limits, the Plummer profile, error trends)
cannot tell a cube of side 2l from one of side l, or (l/r)^3 from (l/r)^2.
Each case here places a handful of particles on the integer grid so that
exactly one node's fate is in question, and reads that fate from the
interaction counts: an accepted node is one particle-node interaction, an
opened leaf is one particle-particle interaction per particle in it.

Paper passages: Sec. "Tree walk and opening criterion" (relative criterion,
eq. eqnrelcriterion; the exclusion region of side 2l around the node's
geometric centre), Sec. "Gravitational softening" (nodes closer than the
softening length are opened), Sec. "TreePM approach" (nodes beyond r_cut are
dropped), Sec. "Fast multipole method" (node pairs that touch never
interact), and the learned-seed feature list written in the oracle.
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle
import workloads

UNIT = 2.0 ** -32          # periodic box of side 1: physical length of one integer step
P0 = 1 << 31               # lower corner of the parent cube P (aligned at every level >= 1)


# ------------------------------------------------------------------ one-sided walk
def walk_positions(lev_n, offset, spread=1000):
    """Node N (level lev_n, side l) = octant 0 of its parent P, holding two
    particles of mass 1/2 placed symmetrically about N's geometric centre
    (so its centre of mass is that centre); the target (index 2) sits at
    `offset` integer steps from that centre, inside P but outside N.
    With leaf_max 2 the tree is a chain root -> ... -> P, then N (a leaf of
    two) and the target's own leaf.  Returns X, Y, Z (uint32), masses,
    l and the target's distance r from N's centre of mass (physical)."""
    ln = 1 << (32 - lev_n)
    cn = P0 + ln // 2
    dx, dy, dz = offset
    assert max(dx, dy, dz) >= ln // 2 and max(dx, dy, dz) < 3 * ln // 2 and min(dx, dy, dz) >= 0
    X = np.array([cn - spread, cn + spread, cn + dx], np.uint32)
    Y = np.array([cn, cn, cn + dy], np.uint32)
    Z = np.array([cn, cn, cn + dz], np.uint32)
    m = np.array([0.5, 0.5, 1e-3])
    return X, Y, Z, m, ln * UNIT, math.sqrt(dx * dx + dy * dy + dz * dz) * UNIT


def _geometry(lev_n, offset):
    X, Y, Z, m, l, r = walk_positions(lev_n, offset)
    t = oracle.Tree(X, Y, Z, m, True, 1.0, 2)
    level, cell, count, leaf = t.nodes()
    # the node in question exists as described
    k = np.flatnonzero((level == lev_n) & (count == 2))
    assert len(k) == 1 and leaf[k[0]] == 1
    return t, l, r


def _target_counts(t, **kw):
    aseed = kw.pop("aseed", None)
    _, _, cnt = t.walk(targets=[2], aseed=aseed, G=1.0, **kw)
    return tuple(int(v) for v in cnt[0])


OPENED, ACCEPTED, DROPPED = (2, 0), (0, 1), (0, 0)


@pytest.mark.parametrize("lev_n", [4, 9])
def test_exclusion_zone_is_cube_of_side_2l(lev_n):
    """A target at l - 1 grid steps from the node's geometric centre lies in
    the exclusion cube (half side l) and must open the node however large
    theta is; at exactly l steps it lies outside and the node is accepted."""
    ln = 1 << (32 - lev_n)
    geo = dict(criterion=0, theta=1e6, eps0=0.0, exclusion=1)
    t, l, r = _geometry(lev_n, (ln - 1, 0, 0))
    assert _target_counts(t, **geo) == OPENED
    t, l, r = _geometry(lev_n, (ln, 0, 0))
    assert _target_counts(t, **geo) == ACCEPTED
    # the region is a cube, not a sphere of radius l: the corner point at
    # (l-1, l-1, l-1) is sqrt(3) l away yet still inside
    t, l, r = _geometry(lev_n, (ln - 1, ln - 1, ln - 1))
    assert r > 1.7 * l
    assert _target_counts(t, **geo) == OPENED
    t, l, r = _geometry(lev_n, (ln - 1, ln - 1, ln))
    assert _target_counts(t, **geo) == ACCEPTED


@pytest.mark.parametrize("order", [3, 2, 4, 5])
def test_relative_criterion_threshold_and_exponent(order):
    """eq. eqnrelcriterion: accept iff (M/r^2)(l/r)^p < alpha |a| with p the
    expansion order; equality and anything above open.  The threshold alpha
    is computed here from the configuration itself (M = 1, l = 1/16, r =
    1.25 l, |a| = 0.37) and both sides of it are probed."""
    lev_n = 4
    ln = 1 << (32 - lev_n)
    t, l, r = _geometry(lev_n, (ln + ln // 4, 0, 0))
    A = 0.37
    aseed = np.array([1.0, 1.0, A])
    a_crit = 1.0 * l ** order / (A * r ** (order + 2))
    kw = dict(criterion=1, order=order, eps0=0.0, exclusion=1, aseed=aseed)
    assert _target_counts(t, alpha=a_crit * (1 + 1e-7), **kw) == ACCEPTED
    assert _target_counts(t, alpha=a_crit * (1 - 1e-7), **kw) == OPENED


def test_relative_criterion_scales_as_l_cubed():
    """At a fixed distance, doubling the node side moves the alpha threshold
    by 2^3 = 8 for p = 3 (not by 4).  Exclusion is off so that the larger
    node is judged by the criterion alone."""
    d = (1 << 28) + (1 << 26)  # 1.25/16 of the box
    A = 1.0
    aseed = np.array([1.0, 1.0, A])
    kw = dict(criterion=1, order=3, eps0=0.0, exclusion=0, aseed=aseed)
    crit = {}
    for lev_n in (4, 3):
        t, l, r = _geometry(lev_n, (d, 0, 0))
        crit[lev_n] = 1.0 * l ** 3 / (A * r ** 5)
        assert _target_counts(t, alpha=crit[lev_n] * (1 + 1e-7), **kw) == ACCEPTED
        assert _target_counts(t, alpha=crit[lev_n] * (1 - 1e-7), **kw) == OPENED
    assert crit[3] / crit[4] == pytest.approx(8.0, rel=1e-12)
    # the larger node at the smaller node's threshold x 4.5 is still opened
    t, l, r = _geometry(3, (d, 0, 0))
    assert _target_counts(t, alpha=crit[4] * 4.5, **kw) == OPENED


def test_nodes_closer_than_softening_edge_are_opened():
    """Softened nodes: a node whose centre of mass is closer than h = 2.8 eps0
    is opened even when the criterion would accept it."""
    ln = 1 << 28
    t, l, r = _geometry(4, (ln + ln // 4, 0, 0))
    geo = dict(criterion=0, theta=1e6, exclusion=1)
    assert _target_counts(t, eps0=r / 2.8 * (1 + 1e-7), **geo) == OPENED
    assert _target_counts(t, eps0=r / 2.8 * (1 - 1e-7), **geo) == ACCEPTED


def test_treepm_drops_nodes_by_nearest_edge_distance():
    """Sec. "TreePM approach": a node whose cube lies entirely beyond r_cut
    (Euclidean distance from the target to the cube's nearest point) is
    skipped; otherwise it is walked as usual."""
    ln = 1 << 28
    kw = dict(kernel=1, r_s=0.01, criterion=0, theta=1e6, eps0=0.0, exclusion=1)
    t, l, r = _geometry(4, (ln + ln // 4, 0, 0))
    e = 0.75 * l  # x-distance from the target to the cube's near face
    assert _target_counts(t, r_cut=e * (1 + 1e-7), **kw) == ACCEPTED
    assert _target_counts(t, r_cut=e * (1 - 1e-7), **kw) == DROPPED
    # diagonal offset: the nearest point is an edge, sqrt(2) x 0.75 l away
    t, l, r = _geometry(4, (ln + ln // 4, ln + ln // 4, 0))
    e2 = math.sqrt(2.0) * 0.75 * l
    assert _target_counts(t, r_cut=e2 * (1 + 1e-7), **kw) == ACCEPTED
    assert _target_counts(t, r_cut=0.9 * e2, **kw) == DROPPED


# ------------------------------------------------------------------ FMM
def fmm_positions(cells, lev=5):
    """One particle (mass 1) in each given level-`lev` cell (integer cell
    offsets from the cube at P0), near the cell centre, moved off it by a
    few grid steps that differ from particle to particle.  With leaf_max 1
    every occupied cell at `lev` is a leaf once its parent holds two
    particles."""
    side = 1 << (32 - lev)
    X, Y, Z = [], [], []
    for k, (cx, cy, cz) in enumerate(cells):
        X.append(P0 + cx * side + side // 2 + 4096 * k * k)
        Y.append(P0 + cy * side + side // 2 + 5 * k)
        Z.append(P0 + cz * side + side // 2 + 3 * k)
    X, Y, Z = (np.array(v, np.uint32) for v in (X, Y, Z))
    return X, Y, Z, np.ones(len(X))


def _fmm_line(cells, lev=5):
    X, Y, Z, m = fmm_positions(cells, lev)
    t = oracle.Tree(X, Y, Z, m, True, 1.0, 1)
    level, cell, count, leaf = t.nodes()
    assert np.all(level[leaf == 1] == lev)
    return t


def test_fmm_touching_cells_never_interact():
    """Four single-particle leaves in a row of level-5 cells 0, 1, 2, 3 (cells
    0-1 and 2-3 share a level-4 parent).  With theta huge, every pair of
    cells that share a face is opened down to particles (3 particle pairs),
    and every pair separated by at least one cell is a node-node
    interaction (0-2, 0-3, 1-3)."""
    t = _fmm_line([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    _, _, st = t.fmm(kernel=0, theta=1e6, eps0=0.0)
    assert tuple(int(v) for v in st) == (3, 0, 3)


def test_fmm_corner_touching_cells_never_interact():
    """Two leaves that meet only at a corner still touch."""
    t = _fmm_line([(0, 0, 0), (1, 1, 1)])
    _, _, st = t.fmm(kernel=0, theta=1e6, eps0=0.0)
    assert tuple(int(v) for v in st) == (1, 0, 0)
    # and a pair one cell apart along every axis does not touch
    t = _fmm_line([(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 3, 3)])
    _, _, st = t.fmm(kernel=0, theta=1e6, eps0=0.0)
    assert tuple(int(v) for v in st) == (3, 0, 3)


def test_fmm_pairs_closer_than_softening_edge_are_opened():
    """Non-touching cells closer than h = 2.8 eps0 are opened as well."""
    t = _fmm_line([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    _, _, st = t.fmm(kernel=0, theta=1e6, eps0=1.0 / 2.8)  # h = 1 > every separation
    assert tuple(int(v) for v in st) == (6, 0, 0)


def test_fmm_criterion_sums_both_sides():
    """Node pair criterion (l_A + l_B)/r < theta: cells 0 and 2 of side l with
    centres of mass 2l apart (up to a few grid steps) interact for theta
    just above (l + l)/r and are opened just below."""
    t = _fmm_line([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    side = 2.0 ** -5
    X, Y, Z = t.X.astype(np.float64), t.Y.astype(np.float64), t.Z.astype(np.float64)
    r02 = math.sqrt((X[2] - X[0]) ** 2 + (Y[2] - Y[0]) ** 2 + (Z[2] - Z[0]) ** 2) * UNIT
    r13 = math.sqrt((X[3] - X[1]) ** 2 + (Y[3] - Y[1]) ** 2 + (Z[3] - Z[1]) ** 2) * UNIT
    r03 = math.sqrt((X[3] - X[0]) ** 2 + (Y[3] - Y[0]) ** 2 + (Z[3] - Z[0]) ** 2) * UNIT
    th = 2 * side / min(r02, r13)
    assert th < 2 * side / r03 * 1.6
    _, _, st = t.fmm(kernel=0, theta=th * (1 + 1e-6), eps0=0.0)
    assert int(st[2]) == 3
    # below the larger of the two thresholds the pair with the smaller r opens
    thr = sorted([2 * side / r02, 2 * side / r13])
    _, _, st = t.fmm(kernel=0, theta=thr[1] * (1 - 1e-6), eps0=0.0)
    assert int(st[2]) == 2 and int(st[0]) == 4


def _fmm_relative_thresholds(t, m, aseed):
    """alpha at which each non-touching pair of the four-cell line switches:
    the relative node-node criterion (M_max / r^2)(l_max / r)^(p-1) < alpha |a|_min
    at p = 3, written out from the positions (l = the level-5 side)."""
    side = 2.0 ** -5
    X, Y, Z = t.X.astype(np.float64), t.Y.astype(np.float64), t.Z.astype(np.float64)
    out = {}
    for a, b in ((0, 2), (0, 3), (1, 3)):
        r = math.sqrt((X[b] - X[a]) ** 2 + (Y[b] - Y[a]) ** 2 + (Z[b] - Z[a]) ** 2) * UNIT
        out[(a, b)] = max(m[a], m[b]) * side ** 2 / (min(aseed[a], aseed[b]) * r ** 4)
    return out


def test_fmm_relative_criterion_threshold():
    """Four single-particle leaves in a row (masses and |a| all different):
    every non-touching pair becomes a node-node interaction exactly when alpha
    passes M_max l_max^2 / (|a|_min r^4), probed at 1 +- 1e-6 of each pair's
    threshold; the touching pairs stay particle pairs.  The thresholds differ
    by factors of 2-10, so a wrong power of l or r, the sum instead of the
    maximum of the masses, or the larger instead of the smaller |a| moves
    every switch."""
    X, Y, Z, _ = fmm_positions([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    m = np.array([1.0, 2.0, 3.0, 0.5])
    aseed = np.array([5.0, 0.7, 3.0, 2.0])
    t = oracle.Tree(X, Y, Z, m, True, 1.0, 1)
    thr = _fmm_relative_thresholds(t, m, aseed)
    vals = sorted(thr.values())
    assert vals[1] / vals[0] > 1.5 and vals[2] / vals[1] > 1.5
    for k, a in enumerate(vals):
        _, _, st = t.fmm(kernel=0, eps0=0.0, criterion=1, alpha=a * (1 + 1e-6), aseed=aseed)
        assert int(st[2]) == k + 1, (k, st)
        _, _, st = t.fmm(kernel=0, eps0=0.0, criterion=1, alpha=a * (1 - 1e-6), aseed=aseed)
        assert int(st[2]) == k, (k, st)
    _, _, st = t.fmm(kernel=0, eps0=0.0, criterion=1, alpha=vals[-1] * 2, aseed=aseed)
    assert tuple(int(v) for v in st) == (3, 0, 3)


def test_fmm_relative_criterion_uses_the_smallest_a_of_either_node():
    """Lowering one particle's |a| fourfold delays the switch of every pair
    that holds it by the same factor (|a|_min is the smaller of the two
    nodes' minima), and only of those pairs."""
    X, Y, Z, _ = fmm_positions([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    m = np.ones(4)
    base = np.full(4, 2.0)
    t = oracle.Tree(X, Y, Z, m, True, 1.0, 1)
    thr = _fmm_relative_thresholds(t, m, base)
    a03 = thr[(0, 3)]
    _, _, st = t.fmm(kernel=0, eps0=0.0, criterion=1, alpha=a03 * 1.01, aseed=base)
    n_before = int(st[2])
    low = base.copy()
    low[3] = 0.5                      # |a|_min of pair (0, 3) and (1, 3) drops 4x
    _, _, st = t.fmm(kernel=0, eps0=0.0, criterion=1, alpha=a03 * 1.01, aseed=low)
    assert int(st[2]) < n_before
    _, _, st = t.fmm(kernel=0, eps0=0.0, criterion=1, alpha=a03 * 4.04, aseed=low)
    assert int(st[2]) >= n_before


# ------------------------------------------------------------------ learned-seed features
def _features_by_definition(X, Y, Z, m, B, kernel, eps0, r_s):
    """The eight seed features of every particle, recomputed in NumPy from
    the node set of a periodic tree (a node exists iff the root, or its parent
    holds more than B particles; pinned separately) and direct sums:
    log10 M_L, log10 l_L, level of L, log10(|x - s_L|/l_L + 1e-3),
    log10(|x - s_P|/l_P + 1e-3), log10 M_P, log10 M_Q and log10 |a_near|,
    with L the particle's leaf, P its parent, Q its grandparent (a missing
    ancestor is replaced by the next node below it) and a_near the pair
    forces of the other particles of L plus point masses at the centres of
    mass of the other children of P and of Q."""
    n = len(X)
    C = np.stack([X, Y, Z], 1).astype(np.int64)
    counts = {}
    for lev in range(22):
        cells = C >> (32 - lev)
        keys, cnt = np.unique(cells, axis=0, return_counts=True)
        for k, c in zip(map(tuple, keys), cnt):
            counts[(lev,) + k] = int(c)

    def exists(node):
        lev = node[0]
        if lev == 0:
            return True
        parent = (lev - 1,) + tuple(v >> 1 for v in node[1:])
        return exists(parent) and counts[parent] > B

    def members(node):
        lev = node[0]
        return np.flatnonzero(np.all((C >> (32 - lev)) == np.array(node[1:]), axis=1))

    def gcentre(node):
        lev = node[0]
        side = 1 << (32 - lev)
        return np.array(node[1:], np.int64) * side + side // 2

    def com(node):
        idx = members(node)
        g = gcentre(node)
        d = ((C[idx] - g + 2 ** 31) % 2 ** 32 - 2 ** 31) * UNIT
        return g, (m[idx, None] * d).sum(0) / m[idx].sum(), m[idx].sum()

    def pairK(r):
        if kernel == 0:
            return r ** -3.0
        a = 0.5 / r_s
        return (special.erfc(a * r) + 2 * a * r / math.sqrt(math.pi) * math.exp(-a * a * r * r)) / r ** 3

    def children(node):
        lev = node[0]
        out = []
        for k in range(8):
            ch = (lev + 1, 2 * node[1] + (k >> 2 & 1), 2 * node[2] + (k >> 1 & 1), 2 * node[3] + (k & 1))
            if ch in counts:
                out.append(ch)
        return out

    assert eps0 == 0.0
    F = np.zeros((n, 8))
    for j in range(n):
        lev = 0
        while lev < 21 and counts[(lev,) + tuple(C[j] >> (32 - lev))] > B:
            lev += 1
        L = (lev,) + tuple(int(v) for v in C[j] >> (32 - lev))
        assert exists(L)
        P = (lev - 1,) + tuple(v >> 1 for v in L[1:]) if lev >= 1 else L
        Q = (lev - 2,) + tuple(v >> 2 for v in L[1:]) if lev >= 2 else P
        gL, sL, ML = com(L)
        gP, sP, MP = com(P)
        _, _, MQ = com(Q)
        lL, lP = 2.0 ** -L[0], 2.0 ** -P[0]
        dL = ((C[j] - gL + 2 ** 31) % 2 ** 32 - 2 ** 31) * UNIT - sL
        dP = ((C[j] - gP + 2 ** 31) % 2 ** 32 - 2 ** 31) * UNIT - sP
        acc = np.zeros(3)
        for k in members(L):
            if k == j:
                continue
            d = ((C[k] - C[j] + 2 ** 31) % 2 ** 32 - 2 ** 31) * UNIT
            acc += m[k] * d * pairK(np.linalg.norm(d))
        for self_, up in ((L, P if lev >= 1 else None), (P, Q if lev >= 2 else None)):
            if up is None:
                break
            for sib in children(up):
                if sib == self_:
                    continue
                g, s, M = com(sib)
                d = ((g - C[j] + 2 ** 31) % 2 ** 32 - 2 ** 31) * UNIT + s
                acc += M * d * pairK(np.linalg.norm(d))
        F[j] = [math.log10(ML), math.log10(lL), L[0], math.log10(np.linalg.norm(dL) / lL + 1e-3),
                math.log10(np.linalg.norm(dP) / lP + 1e-3), math.log10(MP), math.log10(MQ),
                math.log10(max(np.linalg.norm(acc), 1e-30))]
    return F


@pytest.mark.parametrize("kernel", [0, 1])
def test_seed_features_by_definition(kernel):
    ps = workloads.clustered_box(240, seed=71, nhalo=3)
    _, X, Y, Z = oracle.quantize(ps.pos, True, 1.0)
    m = ps.mass * (1.0 + 0.5 * np.sin(np.arange(len(X))))  # unequal masses
    B = 4
    t = oracle.Tree(X, Y, Z, m, True, 1.0, B)
    level, _, _, leaf = t.nodes()
    assert level[leaf == 1].max() >= 4 and level[leaf == 1].min() <= 3  # several levels of leaves
    got = t.features(kernel=kernel, eps0=0.0, r_s=0.02)
    ref = _features_by_definition(X, Y, Z, m, B, kernel, 0.0, 0.02)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)
