"""Plain FP64 oracle of the long-range (particle-mesh) force of TreePM.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; it shares no code
with the HIP library.

Paper passages (Sec. "TreePM approach", Sec. "Periodic boundary conditions"):

* Ewald decomposition of the periodic potential of a unit point mass in a
  cubic box of side L (eq. eqnewal): a real-space sum of erfc(alpha r)/r over
  the images plus a k-space sum over the lattice k = 2 pi n / L, with
  r_s = 1/(2 alpha) and the constant pi/(alpha^2 V).
* The long-range potential (eq. eqnksum) is the k-space sum with the Green's
  function exp(-k^2 r_s^2) / k^2.  Reading: the printed equation omits the
  minus sign that the k-space term carries in eq. eqnewal; the long-range
  potential is attractive like the Newtonian one,
      phi_lr(x) = -G sum_j m_j (4 pi / V) sum_{k != 0} exp(-k^2 r_s^2)/k^2 cos(k.(x - x_j)).
* The PM algorithm that evaluates it: clouds-in-cell (CIC) assignment of the
  masses to an N_g^3 mesh, a discrete Fourier transform, multiplication with
  the Green's function, deconvolution of the assignment and of the
  interpolation (a division by the CIC window, a squared sinc per axis, once
  for each), the inverse transform, a 4th-order finite-difference gradient on
  the mesh, and CIC interpolation of the mesh forces to the particles.

Conventions: mesh points at x_c = c h, h = L / N_g, c = 0 .. N_g - 1; CIC gives
a particle at u = x / h the weights (1 - f) and f on the points floor(u) and
floor(u) + 1 (periodic) per axis, f = u - floor(u).  Positions may be given
as 32-bit integer coordinates (x = X L / 2^32), which makes the cell index and
the weight exact when N_g is a power of two.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


# ---------------------------------------------------------------- exact sums
def kvectors(L: float, r_s: float, kcut: float = 6.0):
    """Lattice vectors k = 2 pi n / L, n != 0, with |k| r_s <= kcut (all signs)."""
    nmax = int(math.ceil(kcut / r_s * L / (2 * math.pi)))
    r = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    n = n[np.any(n != 0, axis=1)]
    k = 2 * math.pi / L * n
    k2 = (k * k).sum(1)
    keep = k2 * r_s * r_s <= kcut * kcut
    return k[keep], k2[keep]


def ewald_long_range(targets, sources, mass, L, r_s, G=1.0, kcut=6.0, chunk=4096):
    """Exact long-range acceleration and potential (the k-space sum of eq.
    eqnksum with the sign of eq. eqnewal) at `targets` (m x 3) from point
    masses at `sources` (n x 3), by the structure factor S(k) = sum_j m_j
    exp(-i k.x_j) over every k with |k| r_s <= kcut (the Green's function is
    below exp(-kcut^2) ~ 2e-16 of its k -> 0 value beyond)."""
    k, k2 = kvectors(L, r_s, kcut)
    g = np.exp(-k2 * r_s * r_s) / k2
    V = L ** 3
    S = np.zeros(len(k), complex)
    for a in range(0, len(sources), chunk):
        S += (mass[a:a + chunk, None] * np.exp(-1j * sources[a:a + chunk] @ k.T)).sum(0)
    acc = np.zeros((len(targets), 3))
    pot = np.zeros(len(targets))
    for a in range(0, len(targets), chunk):
        e = np.exp(1j * targets[a:a + chunk] @ k.T) * S[None, :]   # sum_j m_j exp(i k.(x - x_j))
        # phi = -G (4 pi / V) sum_k g cos(k.d);  a = -grad phi = -G (4 pi / V) sum_k g k sin(k.d)
        pot[a:a + chunk] = -G * 4 * math.pi / V * (e.real * g).sum(1)
        acc[a:a + chunk] = -G * 4 * math.pi / V * (e.imag * g) @ k
    return acc, pot


def ewald_real_space(d, L, r_s, nimg=2):
    """Real-space Ewald sum for one unit mass at separation vectors d (m x 3):
    acceleration sum_q -(d + q) [erfc(a r) + (2 a r / sqrt(pi)) exp(-a^2 r^2)] / r^3
    (pointing at the mass) and potential -sum_q erfc(a r) / r, a = 1/(2 r_s),
    over the images q = L n, |n_i| <= nimg."""
    a = 0.5 / r_s
    acc = np.zeros_like(d)
    pot = np.zeros(len(d))
    r1 = np.arange(-nimg, nimg + 1)
    for n in np.stack(np.meshgrid(r1, r1, r1, indexing="ij"), -1).reshape(-1, 3):
        v = d + L * n
        r = np.linalg.norm(v, axis=1)
        f = (special.erfc(a * r) + 2 * a * r / math.sqrt(math.pi) * np.exp(-a * a * r * r)) / r ** 3
        acc -= v * f[:, None]
        pot -= special.erfc(a * r) / r
    return acc, pot


def madelung_correction(L, r_s, kcut=7.0, nimg=3):
    """psi(0) of eq. eqnewal: 1/r minus the periodic potential of a unit mass
    with neutralising background, as r -> 0:
    psi(0) = 2 a / sqrt(pi) + pi / (a^2 V) - sum_{q != 0} erfc(a q)/q - (4 pi / V) sum_{k != 0} g(k)."""
    a = 0.5 / r_s
    V = L ** 3
    r1 = np.arange(-nimg, nimg + 1)
    n = np.stack(np.meshgrid(r1, r1, r1, indexing="ij"), -1).reshape(-1, 3)
    n = n[np.any(n != 0, axis=1)]
    q = L * np.linalg.norm(n, axis=1)
    k, k2 = kvectors(L, r_s, kcut)
    return (2 * a / math.sqrt(math.pi) + math.pi / (a * a * V) - (special.erfc(a * q) / q).sum()
            - 4 * math.pi / V * (np.exp(-k2 * r_s * r_s) / k2).sum())


# ---------------------------------------------------------------- PM, step by step
def cic_cells(pos, L, ng):
    """Lower mesh point (n x 3 int) and weight of the upper one (n x 3) per axis."""
    u = np.asarray(pos, np.float64) / L * ng
    i = np.floor(u)
    f = u - i
    return i.astype(np.int64) % ng, f


def cic_cells_int(X, Y, Z, ng):
    """The same from 32-bit integer coordinates, exact for ng a power of two."""
    sh = 32 - int(round(math.log2(ng)))
    assert 1 << (32 - sh) == ng
    C = np.stack([np.asarray(A, np.uint64) for A in (X, Y, Z)], 1)
    i = (C >> np.uint64(sh)).astype(np.int64)
    f = (C & np.uint64((1 << sh) - 1)).astype(np.float64) / float(1 << sh)
    return i, f


def cic_deposit(cells, frac, mass, ng):
    """Mass on the mesh: every particle spreads m over its 8 CIC points."""
    M = np.zeros((ng, ng, ng))
    for dx in (0, 1):
        wx = frac[:, 0] if dx else 1 - frac[:, 0]
        for dy in (0, 1):
            wy = frac[:, 1] if dy else 1 - frac[:, 1]
            for dz in (0, 1):
                wz = frac[:, 2] if dz else 1 - frac[:, 2]
                np.add.at(M, ((cells[:, 0] + dx) % ng, (cells[:, 1] + dy) % ng, (cells[:, 2] + dz) % ng),
                          mass * wx * wy * wz)
    return M


def cic_interpolate(field, cells, frac):
    """Field values at the particles with the same 8-point weights."""
    ng = field.shape[0]
    out = np.zeros(len(cells))
    for dx in (0, 1):
        wx = frac[:, 0] if dx else 1 - frac[:, 0]
        for dy in (0, 1):
            wy = frac[:, 1] if dy else 1 - frac[:, 1]
            for dz in (0, 1):
                wz = frac[:, 2] if dz else 1 - frac[:, 2]
                out += wx * wy * wz * field[(cells[:, 0] + dx) % ng, (cells[:, 1] + dy) % ng, (cells[:, 2] + dz) % ng]
    return out


def green_factor(ng, L, r_s, G=1.0):
    """Multiplier of the mesh-mass transform (numpy's full complex FFT layout)
    that gives the mesh potential after numpy's inverse transform:
    -G (4 pi / V) exp(-k^2 r_s^2) / k^2 / W(k)^2 * ng^3, W = prod_i sinc^2(k_i h / 2),
    zero at k = 0."""
    n = np.fft.fftfreq(ng, d=1.0 / ng)  # 0, 1, .., ng/2 - 1, -ng/2, .., -1
    k1 = 2 * math.pi / L * n
    h = L / ng
    s = np.sinc(k1 * h / 2 / math.pi) ** 2  # numpy sinc(x) = sin(pi x)/(pi x)
    kx, ky, kz = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    W = s[:, None, None] * s[None, :, None] * s[None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        f = -G * 4 * math.pi / L ** 3 * np.exp(-k2 * r_s * r_s) / k2 / (W * W) * ng ** 3
    f[0, 0, 0] = 0.0
    return f


def fd4_gradient(phi, axis, h):
    """4th-order central difference: d phi / dx ~ [2/3 (phi_+1 - phi_-1) - 1/12 (phi_+2 - phi_-2)] / h."""
    p1, m1 = np.roll(phi, -1, axis), np.roll(phi, 1, axis)
    p2, m2 = np.roll(phi, -2, axis), np.roll(phi, 2, axis)
    return (2.0 / 3.0 * (p1 - m1) - 1.0 / 12.0 * (p2 - m2)) / h


def pm_long_range(cells, frac, mass, ng, L, r_s, G=1.0, want_pot=False):
    """Long-range accelerations (n x 3) of the particles by the PM steps above
    (and the interpolated mesh potential if asked)."""
    M = cic_deposit(cells, frac, mass, ng)
    phi = np.fft.ifftn(np.fft.fftn(M) * green_factor(ng, L, r_s, G)).real
    h = L / ng
    acc = np.stack([cic_interpolate(-fd4_gradient(phi, a, h), cells, frac) for a in range(3)], 1)
    if want_pot:
        return acc, cic_interpolate(phi, cells, frac)
    return acc
