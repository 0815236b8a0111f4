"""Pins of the hierarchical time-integration oracle (Sec. "Hierarchical time
integration") against what the scheme and mechanics fix."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import kdk


def _plummer(n, seed):
    ps = workloads.plummer(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    vel = 0.3 * rng.normal(size=(n, 3))
    vel -= (ps.mass[:, None] * vel).sum(0) / ps.mass.sum()
    return ps.pos.copy(), vel, ps.mass.copy()


ROOT = (np.array([-40.0, -40.0, -40.0]), 80.0)


def test_without_split_it_is_kick_drift_kick():
    """If no particle needs a step below dt, the step is one leapfrog KDK."""
    pos, vel, m = _plummer(64, 3)
    force = kdk.direct_force(m, eps0=0.05, root=ROOT)
    idx = np.arange(64)
    a0 = force(idx, pos)
    dt = 1e-4
    assert np.all(kdk.timestep(a0, 0.025, 0.05) >= dt)
    p1, v1 = pos.copy(), vel.copy()
    kdk.hierarchical_step(idx, dt, a0, p1, v1, force, 0.025, 0.05)
    # textbook kick-drift-kick, written out here
    p2, v2 = pos.copy(), vel.copy()
    v2 += 0.5 * dt * a0
    p2 += dt * v2
    v2 += 0.5 * dt * force(idx, p2)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v1, v2, rtol=0, atol=1e-15)


def test_uncoupled_subsystems_integrate_independently():
    """Two groups farther apart than the reach of the short-range kernel exert
    no force on each other: the hierarchical step of the union must equal the
    two groups' own hierarchical steps (the slow group a plain KDK step, the
    fast one its own nested sub-steps), to round-off."""
    rng = np.random.default_rng(5)
    L, r_s = 1.0, 0.01
    slow = 0.2 + 0.05 * rng.uniform(size=(40, 3))                  # loose group
    fast = 0.7 + 0.004 * rng.normal(size=(40, 3))                  # tight clump, far beyond 12 r_s
    pos = np.concatenate([slow, fast])
    vel = 0.01 * rng.normal(size=pos.shape)
    m = np.full(80, 1.0 / 80)
    eps = 2e-4
    force = kdk.direct_force(m, eps0=eps, kernel=1, r_s=r_s, box=L)
    idx = np.arange(80)
    a = force(idx, pos)
    dts = kdk.timestep(a, 0.025, eps)
    dt = float(np.min(dts[:40]))                                   # every slow particle is slow
    assert np.all(dts[:40] >= dt) and np.sum(dts[40:] < dt / 2) > 5  # the clump needs two levels or more
    p1, v1 = pos.copy(), vel.copy()
    c1 = kdk.Counter()
    kdk.hierarchical_step(idx, dt, a, p1, v1, force, 0.025, eps, box=L, count=c1)
    p2, v2 = pos.copy(), vel.copy()
    A, B = idx[:40], idx[40:]
    kdk.hierarchical_step(A, dt, force(A, p2), p2, v2, force, 0.025, eps, box=L)
    kdk.hierarchical_step(B, dt, force(B, p2), p2, v2, force, 0.025, eps, box=L)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-13)
    np.testing.assert_allclose(v1, v2, rtol=1e-12, atol=1e-12 * np.abs(v1).max())
    assert max(lv for lv, _ in c1.calls) >= 2


def test_momentum_is_conserved_to_round_off():
    """Every kick applies forces sourced by the set it acts on, so with
    antisymmetric pair forces the total momentum does not change."""
    pos, vel, m = _plummer(200, 7)
    eps = 0.02
    force = kdk.direct_force(m, eps0=eps, root=ROOT)
    idx = np.arange(200)
    a = force(idx, pos)
    p0 = (m[:, None] * vel).sum(0)
    levels = []
    for _ in range(3):
        c = kdk.Counter()
        a = kdk.hierarchical_step(idx, 0.05, a, pos, vel, force, 0.025, eps, count=c)
        levels.append(max(lv for lv, _ in c.calls))
    assert max(levels) >= 2
    dp = np.abs((m[:, None] * vel).sum(0) - p0).max()
    assert dp < 1e-14 * (m[:, None] * np.abs(vel)).sum()


def test_energy_conservation_plummer():
    """A softened Plummer sphere integrated over about two crossing times keeps
    its total energy to a small relative error, and the error falls about
    fourfold when every step is halved (eta / 4 halves the criterion's steps,
    dt_max / 2): second order.  A sign error in any kick or a wrong sub-step
    length breaks this at once."""
    n = 256
    ps = workloads.plummer(n, seed=11)
    rng = np.random.default_rng(12)
    # velocities near virial equilibrium: isotropic, sigma^2 ~ |phi|/6
    org, side = ROOT
    eps = 0.02
    st, X, Y, Z = oracle.quantize(ps.pos, False, side, org)
    _, pot = oracle.direct(X, Y, Z, ps.mass, side / 2.0 ** 31, eps0=eps)
    vel = rng.normal(size=(n, 3)) * np.sqrt(np.abs(pot) / 6.0)[:, None]
    vel -= (ps.mass[:, None] * vel).sum(0)
    pos, m = ps.pos.copy(), ps.mass.copy()
    force = kdk.direct_force(m, eps0=eps, root=ROOT)

    def energy():
        st, X, Y, Z = oracle.quantize(pos, False, side, org)
        _, phi = oracle.direct(X, Y, Z, m, side / 2.0 ** 31, eps0=eps)
        return 0.5 * (m * (vel ** 2).sum(1)).sum() + 0.5 * (m * phi).sum()

    idx = np.arange(n)
    e0 = energy()
    p_init, v_init = pos.copy(), vel.copy()
    err = []
    for eta, dt, steps in ((0.025, 0.1, 20), (0.025 / 4, 0.05, 40)):
        pos[:], vel[:] = p_init, v_init
        a = force(idx, pos)
        for _ in range(steps):
            a = kdk.hierarchical_step(idx, dt, a, pos, vel, force, eta, eps)
        err.append(abs(energy() - e0) / abs(e0))
    assert err[0] < 5e-3 and err[0] / err[1] > 2.5, err


def test_force_count_two_levels():
    """With one fast level the step costs N_0 + 3 N_1 force evaluations (the
    paper's K_hierarchical)."""
    pos, vel, m = _plummer(100, 13)
    eps = 0.02
    force = kdk.direct_force(m, eps0=eps, root=ROOT)
    idx = np.arange(100)
    a = force(idx, pos)
    dts = kdk.timestep(a, 0.025, eps)
    dt = float(np.sort(dts)[70])               # ~30 % fast
    c = kdk.Counter()
    kdk.hierarchical_step(idx, dt, a, pos, vel, force, 0.025, eps, max_level=1, count=c)
    n1 = int(np.sum(dts < dt))
    assert c.evals == kdk.hierarchical_cost([100, n1]) == 100 + 3 * n1
