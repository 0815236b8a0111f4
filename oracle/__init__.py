"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of ``bench.py``
may import this package.  It wraps ``libg4oracle.so`` (built from
``g4oracle.c`` with gcc) through ctypes and shares no code with the HIP
library in ``paper_2010_03567_amd``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "g4oracle.c")
LIB = os.path.join(HERE, "libg4oracle.so")
LIB_NATIVE = os.path.join(HERE, "libg4oracle_native.so")


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc: plain -O2 portable code (tests), or -O3
    -march=native for timing it on the host it runs on."""
    out = LIB_NATIVE if native else LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, out)
    return out


def select(native: bool) -> None:
    """Load the -O3 -march=native build (compiled here, for this host) instead of
    the portable one; call before the first oracle function."""
    global _lib, _which
    if _lib is not None and _which == native:
        return
    if native:
        build(force=True, native=True)
    _lib, _which = None, native


class WalkParams(C.Structure):
    _fields_ = [("kernel", C.c_int), ("criterion", C.c_int), ("order", C.c_int), ("exclusion", C.c_int),
                ("G", C.c_double), ("eps0", C.c_double), ("r_s", C.c_double), ("r_cut", C.c_double),
                ("theta", C.c_double), ("alpha", C.c_double)]


class FmmParams(C.Structure):
    _fields_ = [("kernel", C.c_int), ("G", C.c_double), ("eps0", C.c_double), ("r_s", C.c_double),
                ("r_cut", C.c_double), ("theta", C.c_double), ("criterion", C.c_int), ("alpha", C.c_double)]


_lib = None
_which = False


def lib():
    global _lib
    if _lib is None:
        path = LIB_NATIVE if _which else LIB
        if not os.path.exists(path):
            build(force=True, native=_which)
        L = C.CDLL(path)
        d, p, i64, i32 = C.c_double, C.c_void_p, C.c_int64, C.c_int
        L.orc_soft_K.restype = d; L.orc_soft_K.argtypes = [d, d]
        L.orc_soft_W.restype = d; L.orc_soft_W.argtypes = [d, d]
        L.orc_sr_K.restype = d; L.orc_sr_K.argtypes = [d, d, d]
        L.orc_sr_W.restype = d; L.orc_sr_W.argtypes = [d, d, d]
        L.orc_gn.argtypes = [i32, d, d, p]
        L.orc_Dn.argtypes = [i32, p, d, p, p, p, p]
        L.orc_ewald_psi.argtypes = [p, d, d, p, p, p, p]
        L.orc_gn_ext.argtypes = [i32, d, d, i32, p]
        L.orc_Dfull.argtypes = [p, p, i32, p]
        L.orc_moments4.argtypes = [p]
        L.orc_quantize.restype = i32
        L.orc_quantize.argtypes = [i64, p, i32, d, p, p, p, p]
        L.orc_build.restype = p
        L.orc_build.argtypes = [i64, p, p, p, p, i32, d, i32, i32]
        L.orc_free.argtypes = [p]
        L.orc_tree_nnodes.restype = i64; L.orc_tree_nnodes.argtypes = [p]
        L.orc_tree_nodes.argtypes = [p, p, p, p, p]
        L.orc_moments.argtypes = [p]
        L.orc_build_mt.restype = p
        L.orc_build_mt.argtypes = [i64, p, p, p, p, i32, d, i32, i32, i32]
        L.orc_moments_mt.argtypes = [p, i32]
        L.orc_tree_moments.argtypes = [p, p, p, p, p]
        L.orc_walk.restype = i32
        L.orc_walk.argtypes = [p, C.POINTER(WalkParams), p, p, i64, p, p, p, i32]
        L.orc_direct.argtypes = [i64, p, p, p, p, d, C.POINTER(WalkParams), i32, p, i64, p, p, i32]
        L.orc_fmm.restype = i32
        L.orc_fmm.argtypes = [p, C.POINTER(FmmParams), p, p, p, p]
        L.orc_mlp_forward.argtypes = [p, p, i64, p]
        L.orc_mlp_loss_grad.restype = d
        L.orc_mlp_loss_grad.argtypes = [p, p, p, i64, d, p]
        L.orc_adam.argtypes = [p, p, p, p, i64, d, d, d, d, i64]
        L.orc_two_groups.argtypes = [i64, p, p, i64, p, p, p, p, p, p]
        L.orc_features.restype = i32
        L.orc_features.argtypes = [p, C.POINTER(WalkParams), p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


# ---------------------------------------------------------------- kernels
def soft_K(r, h):
    return lib().orc_soft_K(float(r), float(h))


def soft_W(r, h):
    return lib().orc_soft_W(float(r), float(h))


def sr_K(r, h, alpha):
    return lib().orc_sr_K(float(r), float(h), float(alpha))


def sr_W(r, h, alpha):
    return lib().orc_sr_W(float(r), float(h), float(alpha))


def gn(kernel, r, alpha=0.0):
    g = np.zeros(4)
    lib().orc_gn(int(kernel), float(r), float(alpha), _ptr(g))
    return g


def Dn(kernel, rv, alpha=0.0):
    rv = _f64(rv)
    D0 = np.zeros(1); D1 = np.zeros(3); D2 = np.zeros(9); D3 = np.zeros(27)
    lib().orc_Dn(int(kernel), _ptr(rv), float(alpha), _ptr(D0), _ptr(D1), _ptr(D2), _ptr(D3))
    return D0[0], D1, D2.reshape(3, 3), D3.reshape(3, 3, 3)


# ---------------------------------------------------------------- integers
def quantize(pos, periodic, box, origin=(0.0, 0.0, 0.0)):
    """pos (n,3) float64 -> (status, X, Y, Z) uint32."""
    pos = _f64(pos)
    n = pos.shape[0]
    X = np.zeros(n, np.uint32); Y = np.zeros(n, np.uint32); Z = np.zeros(n, np.uint32)
    org = _f64(origin)
    st = lib().orc_quantize(n, _ptr(pos), int(periodic), float(box), _ptr(org), _ptr(X), _ptr(Y), _ptr(Z))
    return st, X, Y, Z


# ---------------------------------------------------------------- tree
class Tree:
    """Oracle octree over integer positions (recursive index partition)."""

    def __init__(self, X, Y, Z, mass, periodic, box, leaf_max, max_depth=21, nthreads=1):
        self.X, self.Y, self.Z = _u32(X), _u32(Y), _u32(Z)
        self.mass = _f64(mass)
        self.n = self.X.shape[0]
        self.periodic = bool(periodic)
        self.box = float(box)
        self.unit = self.box / (2.0 ** 32 if periodic else 2.0 ** 31)
        if nthreads > 1:
            self._h = lib().orc_build_mt(self.n, _ptr(self.X), _ptr(self.Y), _ptr(self.Z), _ptr(self.mass),
                                         int(periodic), self.box, int(leaf_max), int(max_depth), int(nthreads))
        else:
            self._h = lib().orc_build(self.n, _ptr(self.X), _ptr(self.Y), _ptr(self.Z), _ptr(self.mass),
                                      int(periodic), self.box, int(leaf_max), int(max_depth))
        self.has_moments = False

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    @property
    def nnodes(self):
        return lib().orc_tree_nnodes(self._h)

    def nodes(self):
        m = self.nnodes
        level = np.zeros(m, np.int32); cell = np.zeros((m, 3), np.uint32)
        count = np.zeros(m, np.int64); leaf = np.zeros(m, np.int32)
        lib().orc_tree_nodes(self._h, _ptr(level), _ptr(cell), _ptr(count), _ptr(leaf))
        return level, cell, count, leaf

    def compute_moments(self, nthreads=1):
        lib().orc_moments_mt(self._h, int(nthreads))
        self.has_moments = True

    def moments(self):
        m = self.nnodes
        mass = np.zeros(m); com = np.zeros((m, 3)); q2 = np.zeros((m, 6)); q3 = np.zeros((m, 10))
        lib().orc_tree_moments(self._h, _ptr(mass), _ptr(com), _ptr(q2), _ptr(q3))
        return mass, com, q2, q3

    def walk(self, kernel=0, criterion=0, order=3, exclusion=1, G=1.0, eps0=0.0, r_s=1.0, r_cut=np.inf,
             theta=0.7, alpha=0.005, aseed=None, targets=None, nthreads=1, want_pot=True):
        if not self.has_moments:
            self.compute_moments()
        if order >= 4 and not getattr(self, "has_moments4", False):
            lib().orc_moments4(self._h)
            self.has_moments4 = True
        P = WalkParams(int(kernel), int(criterion), int(order), int(exclusion), float(G), float(eps0),
                       float(r_s), float(r_cut), float(theta), float(alpha))
        tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
        nt = self.n if tg is None else tg.shape[0]
        acc = np.zeros((nt, 3)); pot = np.zeros(nt) if want_pot else None
        cnt = np.zeros((nt, 2), np.int64)
        asd = None if aseed is None else _f64(aseed)
        st = lib().orc_walk(self._h, C.byref(P), _ptr(asd), _ptr(tg), nt, _ptr(acc), _ptr(pot), _ptr(cnt),
                            int(nthreads))
        if st != 0:
            raise RuntimeError(f"orc_walk failed with status {st}")
        return acc, pot, cnt

    def features(self, kernel=0, eps0=0.0, r_s=1.0):
        """Learned-seed features, n x 8 (caller order)."""
        if not self.has_moments:
            self.compute_moments()
        f = np.zeros((self.n, 8))
        P = WalkParams(int(kernel), 0, 3, 1, 1.0, float(eps0), float(r_s), 0.0, 0.0, 0.0)
        if lib().orc_features(self._h, C.byref(P), _ptr(f)) != 0:
            raise RuntimeError("orc_features failed")
        return f

    def fmm(self, kernel=0, G=1.0, eps0=0.0, r_s=1.0, r_cut=np.inf, theta=0.5, criterion=0, alpha=0.005,
            aseed=None):
        """criterion 1: the relative node-node criterion with |a| per particle from aseed."""
        if not self.has_moments:
            self.compute_moments()
        P = FmmParams(int(kernel), float(G), float(eps0), float(r_s), float(r_cut), float(theta), int(criterion),
                      float(alpha))
        asd = None if aseed is None else _f64(aseed)
        acc = np.zeros((self.n, 3)); pot = np.zeros(self.n); st = np.zeros(3, np.int64)
        s = lib().orc_fmm(self._h, C.byref(P), _ptr(asd), _ptr(acc), _ptr(pot), _ptr(st))
        if s != 0:
            raise RuntimeError(f"orc_fmm failed with status {s}")
        return acc, pot, st


def direct(X, Y, Z, mass, unit, kernel=0, G=1.0, eps0=0.0, r_s=1.0, r_cut=np.inf, truncate=False,
           targets=None, nthreads=1):
    X, Y, Z, mass = _u32(X), _u32(Y), _u32(Z), _f64(mass)
    n = X.shape[0]
    P = WalkParams(int(kernel), 0, 3, 1, float(G), float(eps0), float(r_s), float(r_cut), 0.0, 0.0)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    acc = np.zeros((nt, 3)); pot = np.zeros(nt)
    lib().orc_direct(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(mass), float(unit), C.byref(P), int(truncate),
                     _ptr(tg), nt, _ptr(acc), _ptr(pot), int(nthreads))
    return acc, pot


def gn_ext(kernel, r, alpha=0.0, nmax=6):
    """g_0..g_nmax of the Newtonian (kernel 0) or erfc(alpha r)/r (kernel 1) kernel."""
    g = np.zeros(nmax + 1)
    lib().orc_gn_ext(int(kernel), float(r), float(alpha), int(nmax), _ptr(g))
    return g


def d_full(kernel, rv, n, alpha=0.0):
    """The full derivative tensor D_n (shape (3,)*n) of the kernel at offset rv."""
    rv = np.ascontiguousarray(rv, dtype=np.float64)
    g = gn_ext(kernel, float(np.linalg.norm(rv)), alpha, 7)
    D = np.zeros(3 ** n)
    lib().orc_Dfull(_ptr(g), _ptr(rv), int(n), _ptr(D))
    return D.reshape((3,) * n) if n else D[0]


def ewald_psi(x, L=1.0, alpha=0.0):
    """Periodic correction potential psi of a cube of side L (Sec. "Periodic
    boundary conditions", eq. eqnewal) and its derivatives at the points x
    (n x 3): D0 (n,), D1 (n, 3), D2 (n, 3, 3), D3 (n, 3, 3, 3).  alpha <= 0
    selects alpha = 2/L; the result does not depend on alpha."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n = x.shape[0]
    D0 = np.zeros(n); D1 = np.zeros((n, 3)); D2 = np.zeros((n, 3, 3)); D3 = np.zeros((n, 3, 3, 3))
    for q in range(n):
        xq = np.ascontiguousarray(x[q])
        d0 = C.c_double(0.0)
        d1 = np.zeros(3); d2 = np.zeros(9); d3 = np.zeros(27)
        lib().orc_ewald_psi(_ptr(xq), float(L), float(alpha), C.byref(d0), _ptr(d1), _ptr(d2), _ptr(d3))
        D0[q] = d0.value; D1[q] = d1; D2[q] = d2.reshape(3, 3); D3[q] = d3.reshape(3, 3, 3)
    return D0, D1, D2, D3


def two_groups(posA, mA, posB, mB):
    """Forces between two isolated groups: (accA_fmm, accB_fmm, accA_tree, accB_tree)."""
    posA, mA, posB, mB = _f64(posA), _f64(mA), _f64(posB), _f64(mB)
    nA, nB = posA.shape[0], posB.shape[0]
    out = [np.zeros((nA, 3)), np.zeros((nB, 3)), np.zeros((nA, 3)), np.zeros((nB, 3))]
    lib().orc_two_groups(nA, _ptr(posA), _ptr(mA), nB, _ptr(posB), _ptr(mB), *[_ptr(o) for o in out])
    return tuple(out)


# ---------------------------------------------------------------- MLP
NPARAM = 4801


def mlp_forward(w, feat):
    w = _f64(w); feat = _f64(feat)
    n = feat.shape[0]
    out = np.zeros(n)
    lib().orc_mlp_forward(_ptr(w), _ptr(feat), n, _ptr(out))
    return out


def mlp_loss_grad(w, feat, target, tau=0.0):
    w = _f64(w); feat = _f64(feat); target = _f64(target)
    g = np.zeros(NPARAM)
    loss = lib().orc_mlp_loss_grad(_ptr(w), _ptr(feat), _ptr(target), feat.shape[0], float(tau), _ptr(g))
    return loss, g


def adam(w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays w, m, v."""
    lib().orc_adam(_ptr(w), _ptr(_f64(g)), _ptr(m), _ptr(v), w.shape[0], float(lr), float(b1), float(b2),
                   float(eps), int(step))
