"""Plain FP64 oracle of the hierarchical time integration (test infrastructure
only: only the test suite, the smoke check and the benchmark's CPU leg may
import it; it shares no code with the HIP library).

Paper: Sec. "Hierarchical time integration".  A system P with forces sourced
by P itself (known at the start of the step) is split by a timestep criterion
into a slow part S, which the step size dt integrates well enough, and a fast
part F.  The step is the operator sequence

    K_P^P(dt/2)  K_F^F(-dt/2)  E(H_F, dt/2)  D_S(dt)  E(H_F, dt/2)  K_F^F(-dt/2)  K_P^P(dt/2)

(kicks K_A^B apply forces sourced by B to A, D drifts), where E(H_F, dt/2) is
the same step applied recursively to F on its own with half the step size,
and the forces of F sourced by F, computed to split it, are reused as the
starting forces of that recursion.  When F is empty the step is an ordinary
kick-drift-kick.  Every force is sourced by the very set it acts on, so the
scheme conserves momentum when the pairwise forces are antisymmetric.

Timestep criterion (the paper's standard one, Sec. "Time integration of
collisionless particles"): dt_i = sqrt(2 eta eps / |a_i|); a particle is fast
at a level with step dt when dt_i < dt.

Forces come from a callable force(idx, pos) -> acc (the forces on the
particles idx sourced by the particles idx only), so the scheme can be checked
with exact direct sums.
"""
from __future__ import annotations

import numpy as np


class Counter:
    def __init__(self):
        self.evals = 0        # force evaluations (particles that received a force)
        self.calls = []       # (level, size) of every force calculation


def timestep(acc, eta, eps):
    a = np.linalg.norm(acc, axis=1)
    with np.errstate(divide="ignore"):
        return np.where(a > 0, np.sqrt(2 * eta * eps / np.maximum(a, 1e-300)), np.inf)


def hierarchical_step(idx, dt, acc_P, pos, vel, force, eta, eps, box=0.0, level=0, max_level=30, count=None):
    """Advance the particles `idx` (an index array into pos/vel) by dt, given
    their forces acc_P sourced by idx; returns the forces at the end (sourced
    by idx).  pos/vel are updated in place; box > 0 wraps positions into
    [0, box)."""
    count = count if count is not None else Counter()
    dt_i = timestep(acc_P, eta, eps)
    fast = (dt_i < dt) & (level < max_level)
    vel[idx] += 0.5 * dt * acc_P                                   # K_P^P(dt/2)
    if not fast.any():
        drift(idx, dt, pos, vel, box)                              # D_P(dt)
        acc_P = force(idx, pos)
        count.evals += len(idx)
        count.calls.append((level, len(idx)))
        vel[idx] += 0.5 * dt * acc_P                               # K_P^P(dt/2)
        return acc_P
    F, S = idx[fast], idx[~fast]
    acc_F = force(F, pos)
    count.evals += len(F)
    count.calls.append((level + 1, len(F)))
    vel[F] -= 0.5 * dt * acc_F                                     # K_F^F(-dt/2)
    acc_F = hierarchical_step(F, 0.5 * dt, acc_F, pos, vel, force, eta, eps, box, level + 1, max_level, count)
    drift(S, dt, pos, vel, box)                                    # D_S(dt)
    acc_F = hierarchical_step(F, 0.5 * dt, acc_F, pos, vel, force, eta, eps, box, level + 1, max_level, count)
    vel[F] -= 0.5 * dt * acc_F                                     # K_F^F(-dt/2)
    acc_P = force(idx, pos)
    count.evals += len(idx)
    count.calls.append((level, len(idx)))
    vel[idx] += 0.5 * dt * acc_P                                   # K_P^P(dt/2)
    return acc_P


def drift(idx, dt, pos, vel, box):
    pos[idx] += dt * vel[idx]
    if box > 0:
        pos[idx] = np.mod(pos[idx], box)


def leapfrog_step(idx, dt, acc, pos, vel, force, box=0.0):
    """Ordinary kick-drift-kick with one step size (the scheme without a split)."""
    vel[idx] += 0.5 * dt * acc
    drift(idx, dt, pos, vel, box)
    acc = force(idx, pos)
    vel[idx] += 0.5 * dt * acc
    return acc


def direct_force(mass, G=1.0, eps0=0.0, kernel=0, r_s=1.0, box=0.0, root=None):
    """force(idx, pos) by the FP64 direct sum of the C oracle among the
    particles idx, on their 32-bit integer positions (periodic box of side
    `box`, or the isolated root cube `root` = (origin, side))."""
    import oracle

    def force(idx, pos):
        p = pos[idx]
        if box > 0:
            st, X, Y, Z = oracle.quantize(p, True, box)
            unit = box / 2.0 ** 32
        else:
            org, side = root
            st, X, Y, Z = oracle.quantize(p, False, side, org)
            unit = side / 2.0 ** 31
        if st != 0:
            raise RuntimeError("a particle left the root cube")
        acc, _ = oracle.direct(X, Y, Z, mass[idx], unit, kernel=kernel, G=G, eps0=eps0, r_s=r_s, r_cut=np.inf)
        return acc

    return force


def hierarchical_cost(levels_counts):
    """Force evaluations per step predicted for nested bins (the paper's
    K_hierarchical = N_0 + 3 sum_k 2^(k-1) N_k): levels_counts[k] = N_k."""
    n = list(levels_counts)
    return n[0] + 3 * sum(2 ** (k - 1) * n[k] for k in range(1, len(n)))
