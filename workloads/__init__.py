"""Seeded synthetic particle sets standing in for the paper's workloads.

This module only draws random inputs (NumPy ``default_rng``); it holds none of
the solver's arithmetic and is shared by the oracle-side tests and the HIP-side
tests and benchmark.  The cosmological initial conditions and haloes the paper
measures on are not available, so these generators stand in for them:

* ``plummer``        isolated Plummer sphere (the isolated-halo tests of the
                     paper's Sec. "Force errors for an isolated particle
                     distribution" use a Hernquist halo; a Plummer sphere has a
                     closed-form enclosed mass and acceleration);
* ``clustered_box``  periodic box: a fraction of the mass in Hernquist haloes
                     with a power-law mass function, the rest uniform (stands
                     in for the clustered cosmological boxes at z = 0);
* ``forest``         many independent clustered boxes of uneven particle count.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PLUMMER_MASS_FRACTION_R20 = 20.0 ** 3 / (1.0 + 20.0 ** 2) ** 1.5  # M(<20)/M for b = 1


@dataclass
class ParticleSet:
    pos: np.ndarray      # (n, 3) float64
    mass: np.ndarray     # (n,) float64
    box: float           # periodic box side, or 0 for isolated
    meta: dict


def _isotropic(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v


def plummer(n: int = 8192, seed: int = 1, b: float = 1.0, rmax: float = 20.0) -> ParticleSet:
    """Plummer sphere, total mass 1, scale radius b, radii truncated at rmax.

    The radius follows from inverting M(<r)/M = r^3/(r^2+b^2)^{3/2} for a
    uniform mass fraction U in (0, M(<rmax)/M)."""
    rng = np.random.default_rng(seed)
    umax = (rmax / b) ** 3 / (1.0 + (rmax / b) ** 2) ** 1.5
    u = rng.uniform(0.0, umax, size=n)
    r = b / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    mass = np.full(n, 1.0 / n)
    return ParticleSet(pos, mass, 0.0, dict(kind="plummer", n=n, seed=seed, b=b, rmax=rmax))


def halo_masses(rng, nhalo: int, total: float, slope: float = 1.9, decades: float = 3.0) -> np.ndarray:
    """Halo masses with dN/dM ~ M^-slope over `decades` decades, rescaled to sum to `total`."""
    x0, x1 = 1.0, 10.0 ** decades
    e = 1.0 - slope
    u = rng.uniform(size=nhalo)
    x = (x0 ** e + u * (x1 ** e - x0 ** e)) ** (1.0 / e)
    return x * (total / x.sum())


def clustered_box(n: int = 128 ** 3, seed: int = 2, box: float = 1.0, nhalo: int = 2000,
                  halo_fraction: float = 0.6, conc_spread: float = 1.0, slope: float = 1.9,
                  decades: float = 3.0) -> ParticleSet:
    """Periodic box of n equal-mass particles (total mass 1).

    A fraction `halo_fraction` of the particles sits in `nhalo` Hernquist
    haloes with masses dN/dM ~ M^-1.9 over three decades and centres uniform in
    the box; each halo is truncated at r200 (mean enclosed density 200 times the
    box mean) and has scale length a = 0.3 r200 times a factor drawn
    log-uniformly in [spread^-1/2, spread^1/2].  The remaining particles are
    uniform in the box.  Positions are wrapped into [0, box)."""
    rng = np.random.default_rng(seed)
    mp = 1.0 / n
    Mh = halo_masses(rng, nhalo, halo_fraction, slope, decades)
    nh = np.floor(Mh / mp).astype(np.int64)
    nbg = n - int(nh.sum())
    rho_mean = 1.0 / box ** 3
    r200 = (3.0 * Mh / (800.0 * math.pi * rho_mean)) ** (1.0 / 3.0)
    f = np.exp(rng.uniform(-0.5, 0.5, size=nhalo) * math.log(conc_spread)) if conc_spread > 1.0 else np.ones(nhalo)
    a = 0.3 * r200 * f
    centres = rng.uniform(0.0, box, size=(nhalo, 3))
    hid = np.repeat(np.arange(nhalo), nh)
    # Hernquist: M(<r)/M = r^2/(r+a)^2  ->  r = a sqrt(U) / (1 - sqrt(U)), U < (r200/(r200+a))^2
    umax = (r200 / (r200 + a)) ** 2
    u = rng.uniform(size=hid.shape[0]) * umax[hid]
    su = np.sqrt(u)
    r = a[hid] * su / (1.0 - su)
    halo_pos = centres[hid] + r[:, None] * _isotropic(rng, hid.shape[0])
    bg = rng.uniform(0.0, box, size=(nbg, 3))
    pos = np.concatenate([halo_pos, bg], axis=0)
    pos = np.mod(pos, box)
    pos[pos >= box] = 0.0
    perm = rng.permutation(n)  # no ordering hint for the solver
    pos = np.ascontiguousarray(pos[perm])
    mass = np.full(n, mp)
    return ParticleSet(pos, mass, box, dict(kind="clustered_box", n=n, seed=seed, nhalo=nhalo,
                                            halo_fraction=halo_fraction, conc_spread=conc_spread,
                                            n_background=nbg))


def forest_sizes(nbox: int = 64, seed: int = 3000, nmin: int = 32768, nmax: int = 1048576) -> np.ndarray:
    """Box sizes log-uniform in [nmin, nmax]."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=nbox))).astype(np.int64)


def forest(nbox: int = 64, seed: int = 3000, nmin: int = 32768, nmax: int = 1048576, nhalo: int = 2000,
           conc_spread: float = 3.0):
    """Independent clustered boxes (box b uses seed+b); returns a list of ParticleSet.

    The halo count scales with the box size (2000 haloes at 128^3 particles)."""
    sizes = forest_sizes(nbox, seed, nmin, nmax)
    out = []
    for b, nb in enumerate(sizes):
        nh = max(8, int(round(nhalo * nb / 128 ** 3)))
        out.append(clustered_box(int(nb), seed=seed + b, nhalo=nh, conc_spread=conc_spread))
    return out


def sample_indices(n: int, k: int, seed: int = 12345) -> np.ndarray:
    """Sorted random subset of k distinct indices out of n (all if k >= n)."""
    if k >= n:
        return np.arange(n, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def relative_errors(a, a_ref):
    """Per-particle |a - a_ref| / |a_ref| (particles with |a_ref| = 0 dropped)."""
    a = np.asarray(a, dtype=np.float64); a_ref = np.asarray(a_ref, dtype=np.float64)
    nr = np.linalg.norm(a_ref, axis=1)
    ok = nr > 0
    return np.linalg.norm(a[ok] - a_ref[ok], axis=1) / nr[ok]


def percentiles(err, qs=(50, 90, 99, 99.9)):
    return {f"p{q}": float(np.percentile(err, q)) for q in qs}


def isolated_root(pos, margin: float = 1e-3):
    """Shrink-wrapped cubic root for an isolated set: (origin[3], side)."""
    lo = pos.min(axis=0); hi = pos.max(axis=0)
    side = float((hi - lo).max()) * (1.0 + margin)
    if not side > 0.0:  # a single particle (or all coincident): any positive cube holds it
        side = 1.0
    centre = 0.5 * (lo + hi)
    origin = centre - 0.5 * side
    return origin.astype(np.float64), side
