"""Pins of the oracle's periodic correction potential psi (Sec. "Periodic
boundary conditions", eqs. eqnpo1, eqnpo2, eqnewal) and of its periodic
Newtonian + Ewald direct sum and tree walk (kernel 2), against what the paper
and the mathematics fix: the printed psi(0) = 2.8372975/L, independence of the
Ewald split parameter, periodicity of the full Green's function 1/r - psi,
Poisson's equation with the neutralising background, the symmetry points of
the cubic lattice, the small-distance limit, finite differences of the
derivative tensors, and lattice configurations whose forces vanish."""
import numpy as np
import pytest

import oracle


def _psi(x, L=1.0, alpha=0.0):
    return oracle.ewald_psi(np.atleast_2d(x), L, alpha)


def test_psi_at_origin_is_the_printed_constant():
    for L in (1.0, 2.0, 0.37):
        D0, D1, D2, D3 = _psi([0.0, 0.0, 0.0], L)
        assert abs(D0[0] * L - 2.8372975) < 1e-7
        assert np.abs(D1[0]).max() < 1e-12 / L ** 2       # even function: no gradient at 0
        assert np.abs(D3[0]).max() < 1e-10 / L ** 4


def test_independent_of_the_split_parameter():
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.5, 0.5, size=(6, 3))
    ref = _psi(x, 1.0, 2.0)
    for alpha in (1.5, 3.0, 4.0):
        got = _psi(x, 1.0, alpha)
        for a, b in zip(got, ref):
            assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max())


def test_full_greens_function_is_periodic():
    """G(x) = 1/|x| - psi(x) is the sum over all images, so G(x + L n) = G(x)."""
    rng = np.random.default_rng(2)
    x = rng.uniform(-0.5, 0.5, size=(5, 3))

    def G(p):
        D0, D1, _, _ = _psi(p)
        r = np.linalg.norm(p, axis=1)
        return 1.0 / r - D0, -p / r[:, None] ** 3 - D1

    g0, f0 = G(x)
    for shift in ([1, 0, 0], [0, -1, 0], [1, 1, -1]):
        g1, f1 = G(x + np.array(shift, float))
        np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-11)
        np.testing.assert_allclose(f1, f0, rtol=0, atol=1e-10)


def test_poisson_equation_with_background():
    """Inside the cell the image sum obeys lap G = -4 pi delta + 4 pi / V, so
    lap psi = -4 pi / V there and the contracted third derivative vanishes."""
    rng = np.random.default_rng(3)
    for L in (1.0, 3.0):
        x = rng.uniform(-0.45, 0.45, size=(6, 3)) * L
        _, _, D2, D3 = _psi(x, L)
        np.testing.assert_allclose(np.trace(D2, axis1=1, axis2=2), -4 * np.pi / L ** 3, rtol=1e-11)
        np.testing.assert_allclose(np.einsum("nijj->ni", D3), 0.0, atol=1e-10 / L ** 4)


def test_symmetry_points_feel_no_force():
    """A unit mass at d from its own lattice pulls nothing at the cell's face,
    edge and corner centres: grad G = 0 there, i.e. grad psi = -d/|d|^3."""
    pts = np.array([[0.5, 0, 0], [0.5, 0.5, 0], [0.5, 0.5, 0.5], [0, -0.5, 0.5]])
    _, D1, _, _ = _psi(pts)
    r = np.linalg.norm(pts, axis=1)
    np.testing.assert_allclose(D1, -pts / r[:, None] ** 3, rtol=0, atol=1e-11)


def test_cubic_symmetry():
    x = np.array([[0.11, -0.23, 0.37]])
    base = _psi(x)[0][0]
    for y in ([[-0.23, 0.37, 0.11]], [[-0.11, -0.23, 0.37]], [[0.37, 0.11, 0.23]]):
        assert abs(_psi(np.array(y))[0][0] - base) < 1e-13


def test_small_distance_limit():
    """Near the origin psi = psi(0) - (2 pi / 3V) r^2 + O(r^4) (the quadratic
    term is isotropic on the cubic lattice), so grad psi -> -(4 pi / 3V) x with
    a deviation that falls as r^3."""
    u = np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81])
    dev = []
    for r in (0.04, 0.02, 0.01):
        _, D1, _, _ = _psi(r * u)
        dev.append(np.linalg.norm(D1[0] + 4 * np.pi / 3 * r * u))
    assert dev[0] / dev[1] == pytest.approx(8.0, rel=0.05) and dev[1] / dev[2] == pytest.approx(8.0, rel=0.05)
    assert dev[2] < 1e-3 * 4 * np.pi / 3 * 0.01


def test_derivative_tensors_by_finite_differences():
    rng = np.random.default_rng(4)
    h = 1e-4
    for x in rng.uniform(-0.45, 0.45, size=(3, 3)):
        D0, D1, D2, D3 = (a[0] for a in _psi(x))
        for k in range(3):
            e = np.zeros(3); e[k] = h
            p, m = (a[0] for a in _psi(x + e)), (a[0] for a in _psi(x - e))
            p0, p1, p2, _ = p
            m0, m1, m2, _ = m
            assert abs((p0 - m0) / (2 * h) - D1[k]) < 1e-7
            np.testing.assert_allclose((p1 - m1) / (2 * h), D2[:, k], atol=1e-6)
            np.testing.assert_allclose((p2 - m2) / (2 * h), D3[:, :, k], atol=1e-5)
        assert np.allclose(D2, D2.T) and np.allclose(D3, D3.transpose(1, 0, 2)) and np.allclose(D3, D3.transpose(0, 2, 1))


def _lattice(nper, L=1.0):
    g = (np.arange(nper) + 0.25) * (L / nper)
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


def test_direct_sum_on_a_lattice_has_no_forces():
    """Equal masses on a simple cubic lattice: every particle sits at a centre
    of symmetry of the others, so the exact periodic force vanishes; the
    nearest-image Newtonian force alone does not (checked too)."""
    pos = _lattice(2)
    st, X, Y, Z = oracle.quantize(pos, True, 1.0)
    m = np.full(len(pos), 1.0 / len(pos))
    acc, _ = oracle.direct(X, Y, Z, m, 1.0 / 2 ** 32, kernel=2)
    assert np.abs(acc).max() < 1e-12
    pos3 = _lattice(4)         # spacing L/4: exact on the integer grid
    st, X, Y, Z = oracle.quantize(pos3, True, 1.0)
    m3 = np.full(len(pos3), 1.0 / len(pos3))
    acc3, _ = oracle.direct(X, Y, Z, m3, 1.0 / 2 ** 32, kernel=2)
    assert np.abs(acc3).max() < 1e-11
    acc0, _ = oracle.direct(X, Y, Z, m3, 1.0 / 2 ** 32, kernel=0)
    assert np.abs(acc0).max() > 1e-3          # the nearest image alone is not periodic gravity


def test_direct_sum_two_bodies_and_momentum():
    """Two bodies: the force on each is m grad G of the other's offset (the
    full image sum), equal and opposite; many bodies: zero net force."""
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 1, size=(2, 3))
    st, X, Y, Z = oracle.quantize(pos, True, 1.0)
    q = np.stack([X, Y, Z], 1).astype(np.int64)
    d = ((q[1] - q[0] + 2 ** 31) % 2 ** 32 - 2 ** 31) / 2 ** 32
    m = np.array([0.3, 0.7])
    acc, _ = oracle.direct(X, Y, Z, m, 1.0 / 2 ** 32, kernel=2)
    _, D1, _, _ = _psi(d)
    r = np.linalg.norm(d)
    np.testing.assert_allclose(acc[0], m[1] * (d / r ** 3 + D1[0]), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(m[0] * acc[0], -m[1] * acc[1], rtol=1e-12, atol=1e-14)
    pos = rng.uniform(0, 1, size=(40, 3))
    st, X, Y, Z = oracle.quantize(pos, True, 1.0)
    m = rng.uniform(0.5, 1.5, 40)
    acc, _ = oracle.direct(X, Y, Z, m, 1.0 / 2 ** 32, kernel=2, eps0=0.01)
    assert np.abs((m[:, None] * acc).sum(0)).max() < 1e-12 * (m[:, None] * np.abs(acc)).sum()


def test_tree_walk_converges_to_the_ewald_direct_sum():
    """theta -> 0 opens every node down to single particles, so the periodic
    walk equals the Ewald direct sum; at theta = 0.5 the multipole expansion
    of the correction keeps the error small."""
    rng = np.random.default_rng(6)
    n = 300
    pos = np.concatenate([rng.uniform(0, 1, size=(n // 2, 3)),
                          (0.3 + 0.05 * rng.normal(size=(n // 2, 3))) % 1.0])
    m = rng.uniform(0.5, 1.5, n) / n
    st, X, Y, Z = oracle.quantize(pos, True, 1.0)
    ref, _ = oracle.direct(X, Y, Z, m, 1.0 / 2 ** 32, kernel=2, eps0=1e-3, nthreads=8)
    t = oracle.Tree(X, Y, Z, m, True, 1.0, 4)
    exact, _, _ = t.walk(kernel=2, criterion=0, theta=1e-6, eps0=1e-3, nthreads=8)
    np.testing.assert_allclose(exact, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    approx, _, cnt = t.walk(kernel=2, criterion=0, theta=0.5, eps0=1e-3, nthreads=8)
    err = np.linalg.norm(approx - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.median(err) < 2e-3 and cnt[:, 1].sum() > 0


def test_periodic_fmm_with_ewald_correction():
    """The FMM with the Ewald correction in every interaction's expansion:
    theta -> 0 is the Ewald direct sum, the symmetric expansion keeps the
    total momentum at round-off (psi is even, so every correction is
    antisymmetric), and theta = 0.5 stays close to the exact sum."""
    rng = np.random.default_rng(7)
    n = 300
    pos = np.concatenate([rng.uniform(0, 1, size=(n // 2, 3)), (0.3 + 0.05 * rng.normal(size=(n // 2, 3))) % 1.0])
    m = rng.uniform(0.5, 1.5, n) / n
    st, X, Y, Z = oracle.quantize(pos, True, 1.0)
    ref, pref = oracle.direct(X, Y, Z, m, 1.0 / 2 ** 32, kernel=2, eps0=1e-3, nthreads=8)
    t = oracle.Tree(X, Y, Z, m, True, 1.0, 8)
    a0, p0, s0 = t.fmm(kernel=2, theta=1e-9, eps0=1e-3)
    np.testing.assert_allclose(a0, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(p0, pref, rtol=1e-10)
    assert s0[1] == 0 and s0[2] == 0
    a, pa, s1 = t.fmm(kernel=2, theta=0.5, eps0=1e-3)
    assert s1[1] > 0 and s1[2] > 0
    assert np.abs((m[:, None] * a).sum(0)).max() < 1e-13 * (m[:, None] * np.abs(a)).sum()
    err = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.median(err) < 2e-3
    assert np.median(np.abs(pa - pref) / np.abs(pref)) < 1e-3
