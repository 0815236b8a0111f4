"""Pins of the oracle's long-range (PM) force against what the paper and the
mathematics fix: the Madelung-type constant the paper prints, the split
invariance of the Ewald decomposition, the Newtonian limit, exact momentum
conservation of PM, the 4th-order difference operator, CIC's moments, and
convergence of the PM force to the exact k-space sum."""
import math

import numpy as np
import pytest

from oracle import pm


def test_psi_at_origin_is_the_printed_constant():
    """Sec. "Periodic boundary conditions": psi(x -> 0) = 2.8372975 / L for a
    cubic box, whatever split scale the Ewald sum uses."""
    for L in (1.0, 3.0):
        for rs in (0.05 * L, 0.1 * L, 0.2 * L):
            assert pm.madelung_correction(L, rs) * L == pytest.approx(2.8372975, abs=2e-7)


def test_ewald_total_force_is_split_invariant_and_newtonian_up_close():
    """Real-space erfc sum + k-space sum (eqs. eqnewal / eqnksum) is the same
    periodic force for any split scale, and tends to the Newtonian force of
    the mass at small separations (the long-range part's sign and
    normalisation are fixed by this)."""
    rng = np.random.default_rng(3)
    L = 1.0
    d = rng.uniform(-0.5, 0.5, size=(40, 3))
    d[:5] = d[:5] / np.linalg.norm(d[:5], axis=1)[:, None] * 1e-3  # close pairs
    src = np.zeros((1, 3))
    tot = []
    for rs in (0.04, 0.08):
        sr, _ = pm.ewald_real_space(d, L, rs, nimg=2)
        lr, _ = pm.ewald_long_range(d, src, np.ones(1), L, rs)
        tot.append(sr + lr)
    np.testing.assert_allclose(tot[0], tot[1], rtol=1e-9, atol=1e-9)
    newton = -d[:5] / np.linalg.norm(d[:5], axis=1)[:, None] ** 3
    np.testing.assert_allclose(tot[0][:5], newton, rtol=1e-6)


def _system(n=1000, seed=7):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1.0, (n, 3))
    pos[: n // 3] = (0.3 + 0.03 * rng.normal(size=(n // 3, 3))) % 1.0
    return pos, np.full(n, 1.0 / n) * (1 + 0.5 * rng.uniform(size=n))


def test_pm_converges_to_exact_long_range_force():
    """PM against the exact k-space sum at the same split (r_s = 1.25 L/32):
    errors of the long-range force fall about fourfold when the mesh is
    doubled (CIC and the 4th-order gradient are second order at this
    smoothing), and stay at the few-per-mille level the paper's force-law
    figures show for A_smth ~ 1.25."""
    pos, m = _system()
    L, rs = 1.0, 1.25 / 32
    ex, _ = pm.ewald_long_range(pos, pos, m, L, rs, kcut=5.5)
    med = []
    for ng in (32, 64):
        c, f = pm.cic_cells(pos, L, ng)
        a = pm.pm_long_range(c, f, m, ng, L, rs)
        e = np.linalg.norm(a - ex, axis=1) / np.linalg.norm(ex, axis=1)
        med.append(np.median(e))
        assert np.percentile(e, 99) < (6e-2 if ng == 32 else 1.5e-2)
    assert med[0] < 1e-2 and 2.5 < med[0] / med[1] < 6.0


def test_pm_conserves_momentum_and_mass():
    """Same assignment and interpolation, a symmetric Green's function and an
    antisymmetric difference operator: the PM forces sum to zero."""
    pos, m = _system(3000, seed=8)
    c, f = pm.cic_cells(pos, 1.0, 32)
    M = pm.cic_deposit(c, f, m, 32)
    assert M.sum() == pytest.approx(m.sum(), rel=1e-14)
    a = pm.pm_long_range(c, f, m, 32, 1.0, 1.25 / 32)
    net = np.abs((m[:, None] * a).sum(0)).max()
    assert net < 1e-13 * (m[:, None] * np.abs(a)).sum()


def test_cic_centre_of_mass_and_integer_cells():
    """CIC keeps the first moment of each particle (its weights average to its
    position) and the integer-coordinate path gives the same cells and weights."""
    rng = np.random.default_rng(9)
    ng = 16
    X = rng.integers(0, 2 ** 32, size=(500, 3), dtype=np.uint64).astype(np.uint32)
    pos = X.astype(np.float64) / 2.0 ** 32
    c1, f1 = pm.cic_cells(pos, 1.0, ng)
    c2, f2 = pm.cic_cells_int(X[:, 0], X[:, 1], X[:, 2], ng)
    assert np.array_equal(c1, c2)
    np.testing.assert_allclose(f1, f2, rtol=0, atol=1e-15)
    h = 1.0 / ng
    np.testing.assert_allclose(c1 * h + f1 * h, pos, atol=1e-12)


def test_fourth_order_difference_transfer_function():
    """On a single Fourier mode the mesh gradient equals the exact derivative
    times [4/3 sinc(kh) - 1/3 sinc(2kh)] (the 4th-order central difference)."""
    ng, L = 32, 1.0
    h = L / ng
    x = np.arange(ng) * h
    for n in (1, 3, 7):
        k = 2 * math.pi * n / L
        phi = np.broadcast_to(np.sin(k * x)[:, None, None], (ng, ng, ng)).copy()
        got = pm.fd4_gradient(phi, 0, h)[:, 0, 0]
        tf = 4.0 / 3.0 * math.sin(k * h) / (k * h) - 1.0 / 3.0 * math.sin(2 * k * h) / (2 * k * h)
        np.testing.assert_allclose(got, k * np.cos(k * x) * tf, atol=1e-12 * k)
