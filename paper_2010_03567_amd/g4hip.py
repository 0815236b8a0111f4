"""Thin ctypes binding of libg4hip.so (argument marshalling only).

Every function of ``include/g4hip.h`` is exposed under the same name.  Device
arrays are passed as torch CUDA (HIP) tensors; PyTorch provides memory and the
current stream, every step of the solver runs in the library's HIP kernels.
The library must be built (``python -m paper_2010_03567_amd.build``); a
missing library is an ImportError, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libg4hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_03567_amd.build`")

_L = C.CDLL(LIB_PATH)

G4_OK, G4_EINVAL, G4_ENOMEM, G4_EHIP, G4_ESTATE, G4_EROOT = 0, -1, -2, -3, -4, -5


class g4_tree_params(C.Structure):
    _fields_ = [("periodic", C.c_int), ("box", C.c_double), ("origin", C.c_double * 3),
                ("leaf_max", C.c_int), ("max_depth", C.c_int), ("key_kind", C.c_int)]


class g4_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("mass", C.c_void_p)]


class g4_walk_params(C.Structure):
    _fields_ = [("kernel", C.c_int), ("criterion", C.c_int), ("order", C.c_int), ("exclusion", C.c_int),
                ("G", C.c_double), ("eps0", C.c_double), ("r_s", C.c_double), ("r_cut", C.c_double),
                ("theta", C.c_double), ("alpha", C.c_double), ("theta_seed", C.c_double),
                ("a_seed", C.c_void_p), ("group_size", C.c_int), ("seed_from_tree", C.c_int),
                ("sr_table", C.c_int), ("ewald_table", C.c_void_p), ("ewald_n", C.c_int)]


class g4_fmm_params(C.Structure):
    _fields_ = [("kernel", C.c_int), ("G", C.c_double), ("eps0", C.c_double), ("r_s", C.c_double),
                ("r_cut", C.c_double), ("theta", C.c_double), ("deterministic", C.c_int), ("criterion", C.c_int),
                ("alpha", C.c_double), ("a_seed", C.c_void_p), ("ewald_table", C.c_void_p), ("ewald_n", C.c_int)]


class g4_pm_params(C.Structure):
    _fields_ = [("ng", C.c_int), ("r_s", C.c_double), ("G", C.c_double)]


class g4_kdk_params(C.Structure):
    _fields_ = [("solver", C.c_int), ("tp", g4_tree_params), ("wp", g4_walk_params), ("fp", g4_fmm_params),
                ("eta", C.c_double), ("eps", C.c_double), ("max_level", C.c_int)]


class g4_kdk_stats(C.Structure):
    _fields_ = [("force_evals", C.c_uint64), ("force_calls", C.c_uint32), ("deepest_level", C.c_uint32),
                ("evals_per_level", C.c_uint64 * 32)]

    def as_dict(self):
        return {"force_evals": int(self.force_evals), "force_calls": int(self.force_calls),
                "deepest_level": int(self.deepest_level), "evals_per_level": [int(v) for v in self.evals_per_level]}


class g4_stats(C.Structure):
    _fields_ = [("t_build", C.c_double), ("t_moments", C.c_double), ("t_seed", C.c_double),
                ("t_walk", C.c_double),
                ("n_p2p", C.c_uint64), ("n_p2m", C.c_uint64), ("n_visit", C.c_uint64),
                ("n_seed_p2p", C.c_uint64), ("n_seed_p2m", C.c_uint64), ("n_seed_visit", C.c_uint64),
                ("n_pp", C.c_uint64), ("n_pn", C.c_uint64), ("n_nn", C.c_uint64),
                ("n_nodes", C.c_uint64), ("w_pop", C.c_uint64), ("w_p2m", C.c_uint64), ("w_p2p", C.c_uint64),
                ("flags", C.c_uint32), ("max_stack", C.c_uint32),
                ("w_entry", C.c_uint64), ("w_leaf", C.c_uint64), ("w_chunk", C.c_uint64),
                ("n_group_use", C.c_uint64), ("n_group_drop", C.c_uint64)]

    def as_dict(self):
        return {k: (float if k.startswith("t_") else int)(getattr(self, k)) for k, _ in self._fields_}


_p, _i64, _i32, _sz = C.c_void_p, C.c_int64, C.c_int, C.c_size_t
_SIGS = {
    "g4_ctx_create": [_i32, _p, C.POINTER(C.c_void_p)],
    "g4_ctx_destroy": [_p],
    "g4_quantize": [_p, _p, _i64, C.POINTER(g4_tree_params), _p, _p, _p, _p],
    "g4_workspace_bytes": [C.POINTER(g4_tree_params), _i64, C.POINTER(_sz)],
    "g4_build_tree": [_p, C.POINTER(g4_particles), C.POINTER(g4_tree_params), _p, _sz, C.POINTER(C.c_void_p)],
    "g4_compute_multipoles": [_p, _p, _i32],
    "g4_tree_info": [_p, _p, C.POINTER(_i64), _p],
    "g4_tree_export": [_p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p],
    "g4_tree_free": [_p, _p],
    "g4_tree_force": [_p, _p, C.POINTER(g4_walk_params), _p, _p, _p, _p, _p, _p, C.POINTER(g4_stats)],
    "g4_treepm_shortrange": [_p, _p, C.POINTER(g4_walk_params), _p, _p, _p, _p, _p, _p, C.POINTER(g4_stats)],
    "g4_direct_force": [_p, C.POINTER(g4_particles), C.POINTER(g4_tree_params), C.POINTER(g4_walk_params), _i32,
                        _p, _i64, _p, _p, _p, _p],
    "g4_mlp_features": [_p, _p, C.POINTER(g4_walk_params), _p, _p],
    "g4_pm_workspace_bytes": [_i32, C.POINTER(_sz)],
    "g4_kdk_workspace_bytes": [C.POINTER(g4_kdk_params), _i64, C.POINTER(_sz)],
    "g4_kdk_step": [_p, C.POINTER(g4_kdk_params), _i64, _p, _p, _p, C.c_double, _p, _p, _p, _i32, _p, _sz,
                    C.POINTER(g4_kdk_stats)],
    "g4_pm_longrange": [_p, _p, C.POINTER(g4_pm_params), _p, _sz, _i32, _p, _p, _p, _p],
    "g4_ewald_table": [_p, C.c_double, _i32, _p, _sz],
    "g4_compute_moments4": [_p, _p, _p, _sz],
    "g4_ewald_eval": [_p, _p, _i32, C.c_double, _i64, _p, _p, _p, _p, _p, _p, _p],
    "g4_fmm_workspace_bytes": [_p, C.POINTER(g4_fmm_params), C.c_double, C.POINTER(_sz)],
    "g4_forest_workspace_bytes": [C.POINTER(g4_tree_params), _i32, _i64, C.POINTER(_sz)],
    "g4_build_forest": [_p, _i32, _p, C.POINTER(g4_particles), C.POINTER(g4_tree_params), _p, _sz,
                        C.POINTER(C.c_void_p)],
    "g4_fmm_force": [_p, _p, C.POINTER(g4_fmm_params), C.c_double, _p, _sz, _p, _p, _p, _p, C.POINTER(g4_stats)],
    "g4_fmm_force_noalloc": [_p, _p, C.POINTER(g4_fmm_params), _p, _p, _p, _p, C.POINTER(g4_stats)],
    "g4_mlp_forward": [_p, _p, _p, _i64, _p, C.c_float, _i32],
    "g4_mlp_grad": [_p, _p, _p, _p, _i64, C.c_float, _p, _p],
    "g4_mlp_adam": [_p, _p, _p, _p, _p, _p, C.c_float, C.c_float, C.c_float, C.c_float, _i64],
    "g4_mlp_train_step": [_p, _p, _p, _p, _p, _p, _p, _i64, C.c_float, C.c_float, _i64, _p],
}
for _name, _args in _SIGS.items():
    f = getattr(_L, _name)
    f.argtypes = _args
    f.restype = C.c_int
_L.g4_last_error.argtypes = [_p]
_L.g4_last_error.restype = C.c_char_p
_L.g4_ewald_table_bytes.argtypes = [_i32]
_L.g4_ewald_table_bytes.restype = _sz
_L.g4_moments4_bytes.argtypes = [_p]
_L.g4_moments4_bytes.restype = _sz

OPTIONAL_SYMBOLS = []  # filled by extensions below when present


def exported_symbols():
    """Names of the entry points this binding found in the library."""
    return sorted(_SIGS) + ["g4_last_error", "g4_ewald_table_bytes", "g4_moments4_bytes"] + OPTIONAL_SYMBOLS


class G4Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"g4 status {code}: {msg}")
        self.code = code


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


class Context:
    """g4_ctx bound to the current device and torch's current stream."""

    def __init__(self, device=None, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libg4hip needs a HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._check(_L.g4_ctx_create(self.device.index, C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self.h = h

    def _check(self, code, h=None):
        if code != G4_OK:
            msg = _L.g4_last_error(h if h is not None else getattr(self, "h", None))
            raise G4Error(code, msg.decode() if msg else "")

    def check(self, code):
        self._check(code, self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _L is not None:  # module globals may already be gone at interpreter exit
            _L.g4_ctx_destroy(h)
            self.h = None


def tree_params(periodic, box, origin=(0.0, 0.0, 0.0), leaf_max=8, max_depth=21, key_kind=0):
    tp = g4_tree_params()
    tp.periodic = int(periodic)
    tp.box = float(box)
    for k in range(3):
        tp.origin[k] = float(origin[k])
    tp.leaf_max = int(leaf_max)
    tp.max_depth = int(max_depth)
    tp.key_kind = int(key_kind)
    return tp


def walk_params(kernel=0, criterion=0, order=3, exclusion=1, G=1.0, eps0=0.0, r_s=1.0, r_cut=1e30, theta=0.7,
                alpha=0.005, theta_seed=0.7, a_seed=None, group_size=64, seed_from_tree=0, sr_table=0, ewald=None):
    """ewald: the EwaldTable of the box for kernel 2."""
    wp = g4_walk_params()
    wp.kernel, wp.criterion, wp.order, wp.exclusion = int(kernel), int(criterion), int(order), int(exclusion)
    wp.G, wp.eps0, wp.r_s, wp.r_cut = float(G), float(eps0), float(r_s), float(r_cut)
    wp.theta, wp.alpha, wp.theta_seed = float(theta), float(alpha), float(theta_seed)
    wp.a_seed = None if a_seed is None else a_seed.data_ptr()
    wp.group_size = int(group_size)
    wp.seed_from_tree = int(seed_from_tree)
    wp.sr_table = int(sr_table)
    if ewald is not None:
        wp.ewald_table, wp.ewald_n = ewald.ptr, int(ewald.ne)
    wp._keep = (a_seed, ewald)
    return wp


def particles(x, y, z, mass):
    p = g4_particles()
    p.n = x.numel()
    p.x, p.y, p.z, p.mass = x.data_ptr(), y.data_ptr(), z.data_ptr(), mass.data_ptr()
    p._keep = (x, y, z, mass)
    return p


# ------------------------------------------------------------------ calls
def g4_quantize(ctx, pos, tp):
    """pos: (n, 3) float64 device tensor -> (x, y, z) uint32 device tensors (int32 storage)."""
    n = pos.shape[0]
    dev = pos.device
    x = torch.empty(n, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    flag = torch.empty(1, dtype=torch.int32, device=dev)  # cleared by the library when it is used
    ctx.check(_L.g4_quantize(ctx.h, _ptr(pos), n, C.byref(tp), _ptr(x), _ptr(y), _ptr(z), _ptr(flag)))
    return x, y, z


def g4_workspace_bytes(tp, n):
    b = C.c_size_t()
    code = _L.g4_workspace_bytes(C.byref(tp), int(n), C.byref(b))
    if code != G4_OK:
        raise G4Error(code, "workspace size query failed")
    return int(b.value)


class Tree:
    """Handle of a built tree; owns its workspace tensor."""

    def __init__(self, ctx, h, ws, tp, n, parts):
        self.ctx, self.h, self.ws, self.tp, self.n, self._parts = ctx, h, ws, tp, n, parts

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _L is not None:
            _L.g4_tree_free(self.ctx.h, h)
            self.h = None


def g4_build_tree(ctx, p, tp, ws=None):
    nbytes = g4_workspace_bytes(tp, p.n)
    if ws is None:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
    off = (-ws.data_ptr()) % 256
    wsv = ws[off:]
    h = C.c_void_p()
    ctx.check(_L.g4_build_tree(ctx.h, C.byref(p), C.byref(tp), C.c_void_p(wsv.data_ptr()), wsv.numel(), C.byref(h)))
    return Tree(ctx, h, ws, tp, int(p.n), p)


def g4_compute_multipoles(ctx, tree, order=3):
    ctx.check(_L.g4_compute_multipoles(ctx.h, tree.h, int(order)))


def g4_tree_info(ctx, tree):
    nn = C.c_int64()
    ls = (C.c_int64 * (tree.tp.max_depth + 2))()
    ctx.check(_L.g4_tree_info(ctx.h, tree.h, C.byref(nn), C.cast(ls, C.c_void_p)))
    return int(nn.value), list(ls)


def g4_tree_export(ctx, tree, moments=True):
    nn, _ = g4_tree_info(ctx, tree)
    dev = ctx.device
    out = dict(level=torch.empty(nn, dtype=torch.int32, device=dev),
               cell=torch.empty((nn, 3), dtype=torch.int32, device=dev),
               count=torch.empty(nn, dtype=torch.int64, device=dev),
               first=torch.empty(nn, dtype=torch.int64, device=dev),
               leaf=torch.empty(nn, dtype=torch.int32, device=dev))
    if moments:
        out.update(mass=torch.empty(nn, dtype=torch.float64, device=dev),
                   com=torch.empty((nn, 3), dtype=torch.float64, device=dev),
                   q2=torch.empty((nn, 6), dtype=torch.float64, device=dev),
                   q3=torch.empty((nn, 10), dtype=torch.float64, device=dev))
    g = lambda k: _ptr(out[k]) if k in out else None
    ctx.check(_L.g4_tree_export(ctx.h, tree.h, g("level"), g("cell"), g("count"), g("first"), g("leaf"), g("mass"),
                                g("com"), g("q2"), g("q3")))
    return out


def _force_outputs(n, dev, want_pot, want_counts, want_amag):
    ax = torch.empty(n, dtype=torch.float64, device=dev)
    ay = torch.empty_like(ax)
    az = torch.empty_like(ax)
    pot = torch.empty_like(ax) if want_pot else None
    cnt = torch.empty((n, 2), dtype=torch.int32, device=dev) if want_counts else None
    am = torch.empty(n, dtype=torch.float32, device=dev) if want_amag else None
    return ax, ay, az, pot, cnt, am


def g4_tree_force(ctx, tree, wp, want_pot=False, want_counts=False, want_amag=False, want_stats=False, out=None,
                  shortrange=False):
    ax, ay, az, pot, cnt, am = out if out is not None else _force_outputs(tree.n, ctx.device, want_pot, want_counts,
                                                                            want_amag)
    st = g4_stats() if want_stats else None
    fn = _L.g4_treepm_shortrange if shortrange else _L.g4_tree_force
    ctx.check(fn(ctx.h, tree.h, C.byref(wp), _ptr(ax), _ptr(ay), _ptr(az), _ptr(pot), _ptr(cnt), _ptr(am),
                 C.byref(st) if st is not None else None))
    return dict(ax=ax, ay=ay, az=az, pot=pot, counts=cnt, amag=am, stats=st.as_dict() if st is not None else None)


def g4_treepm_shortrange(ctx, tree, wp, **kw):
    return g4_tree_force(ctx, tree, wp, shortrange=True, **kw)


def g4_direct_force(ctx, p, tp, wp, targets=None, truncate=False, want_pot=True):
    nt = p.n if targets is None else targets.numel()
    ax, ay, az, pot, _, _ = _force_outputs(nt, ctx.device, want_pot, False, False)
    ctx.check(_L.g4_direct_force(ctx.h, C.byref(p), C.byref(tp), C.byref(wp), int(truncate), _ptr(targets), int(nt),
                                 _ptr(ax), _ptr(ay), _ptr(az), _ptr(pot)))
    return dict(ax=ax, ay=ay, az=az, pot=pot)


# ------------------------------------------------------------------ PM long range
def pm_params(ng, r_s, G=1.0):
    pp = g4_pm_params()
    pp.ng, pp.r_s, pp.G = int(ng), float(r_s), float(G)
    return pp


def g4_moments4_bytes(tree):
    return int(_L.g4_moments4_bytes(tree.h))


def g4_compute_moments4(ctx, tree, ws=None):
    """Fourth moments of every node (for walks at p = 4, 5) into `ws` (a uint8
    device tensor, allocated when missing or too small); the buffer is kept on
    the tree object."""
    nbytes = int(_L.g4_moments4_bytes(tree.h))
    buf = ws if ws is not None and ws.numel() >= nbytes + 256 else torch.empty(nbytes + 256, dtype=torch.uint8,
                                                                                  device=ctx.device)
    off = (-buf.data_ptr()) % 256
    ctx.check(_L.g4_compute_moments4(ctx.h, tree.h, C.c_void_p(buf.data_ptr() + off), nbytes))
    tree._moments4 = buf
    return buf


class EwaldTable:
    """Device table of the periodic correction potential psi of a cube of side
    `box` (g4_ewald_table); keeps its buffer alive."""

    def __init__(self, ctx, box, ne=32):
        nbytes = int(_L.g4_ewald_table_bytes(int(ne)))
        if nbytes == 0:
            raise G4Error(G4_EINVAL, "ne must be 4..128")
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
        off = (-self.buf.data_ptr()) % 256
        self.ptr = self.buf.data_ptr() + off
        self.box, self.ne, self.nbytes = float(box), int(ne), nbytes
        ctx.check(_L.g4_ewald_table(ctx.h, self.box, self.ne, C.c_void_p(self.ptr), nbytes))

    def values(self):
        """The table as a ((ne+1)^3, 84) float32 tensor (a view)."""
        off = self.ptr - self.buf.data_ptr()
        return self.buf[off:off + self.nbytes].view(torch.float32).view(-1, 84)


def g4_ewald_eval(ctx, table, d):
    """psi and grad psi at offsets d ((n, 3) float64 device tensor) through the
    table's Taylor lookup: returns (psi (n,), grad (n, 3)) float64."""
    n = d.shape[0]
    dx, dy, dz = (d[:, k].contiguous() for k in range(3))
    psi = torch.empty(n, dtype=torch.float64, device=ctx.device)
    g = [torch.empty(n, dtype=torch.float64, device=ctx.device) for _ in range(3)]
    ctx.check(_L.g4_ewald_eval(ctx.h, C.c_void_p(table.ptr), table.ne, table.box, n, _ptr(dx), _ptr(dy), _ptr(dz),
                               _ptr(psi), _ptr(g[0]), _ptr(g[1]), _ptr(g[2])))
    return psi, torch.stack(g, 1)


def g4_pm_workspace_bytes(ng):
    b = C.c_size_t()
    code = _L.g4_pm_workspace_bytes(int(ng), C.byref(b))
    if code != G4_OK:
        raise G4Error(code, "pm workspace size query failed")
    return int(b.value)


def g4_pm_longrange(ctx, tree, pp, ws=None, accumulate=False, want_pot=False, out=None):
    """Long-range TreePM accelerations (and potential); with accumulate they are
    added to `out` (ax, ay, az, pot) instead of written."""
    if out is None:
        ax, ay, az, pot, _, _ = _force_outputs(tree.n, ctx.device, want_pot, False, False)
    else:
        ax, ay, az, pot = out[:4]
    nbytes = g4_pm_workspace_bytes(pp.ng)
    if ws is None or ws.numel() < nbytes + 256:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
    off = (-ws.data_ptr()) % 256
    wsv = ws[off:]
    ctx.check(_L.g4_pm_longrange(ctx.h, tree.h, C.byref(pp), C.c_void_p(wsv.data_ptr()), wsv.numel(),
                                 int(bool(accumulate)), _ptr(ax), _ptr(ay), _ptr(az), _ptr(pot)))
    return dict(ax=ax, ay=ay, az=az, pot=pot, ws=ws)


# ------------------------------------------------------------------ time integration
def kdk_params(solver, tp, eta, eps, max_level=10, wp=None, fp=None):
    kp = g4_kdk_params()
    kp.solver, kp.tp, kp.eta, kp.eps, kp.max_level = int(solver), tp, float(eta), float(eps), int(max_level)
    if wp is not None:
        kp.wp = wp
    if fp is not None:
        kp.fp = fp
    kp._keep = (wp,)
    return kp


def g4_kdk_workspace_bytes(kp, n):
    b = C.c_size_t()
    code = _L.g4_kdk_workspace_bytes(C.byref(kp), int(n), C.byref(b))
    if code != G4_OK:
        raise G4Error(code, "kdk workspace size query failed")
    return int(b.value)


def g4_kdk_step(ctx, kp, pos, vel, mass, dt, acc=None, ws=None):
    """One hierarchical step; pos, vel (n, 3) float64 updated in place; acc:
    (ax, ay, az) float64 tensors holding the forces at the start, or None to
    compute them.  Returns (acc, stats, ws)."""
    n = pos.shape[0]
    have = acc is not None
    if acc is None:
        acc = tuple(torch.empty(n, dtype=torch.float64, device=ctx.device) for _ in range(3))
    nbytes = g4_kdk_workspace_bytes(kp, n)
    if ws is None or ws.numel() < nbytes + 256:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
    off = (-ws.data_ptr()) % 256
    wsv = ws[off:]
    st = g4_kdk_stats()
    ctx.check(_L.g4_kdk_step(ctx.h, C.byref(kp), n, _ptr(pos), _ptr(vel), _ptr(mass), float(dt), _ptr(acc[0]),
                             _ptr(acc[1]), _ptr(acc[2]), int(have), C.c_void_p(wsv.data_ptr()), wsv.numel(),
                             C.byref(st)))
    return acc, st.as_dict(), ws


# ------------------------------------------------------------------ learned seed
MLP_NPARAM = 4801


def g4_mlp_features(ctx, tree, wp, norm=None, out=None):
    feat = out if out is not None else torch.empty((tree.n, 8), dtype=torch.float32, device=ctx.device)
    ctx.check(_L.g4_mlp_features(ctx.h, tree.h, C.byref(wp), _ptr(norm), _ptr(feat)))
    return feat


def g4_mlp_forward(ctx, w_bf16, feat, shift=0.0, mode=0, out=None):
    n = feat.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=ctx.device)
    ctx.check(_L.g4_mlp_forward(ctx.h, _ptr(w_bf16), _ptr(feat), n, _ptr(out), float(shift), int(mode)))
    return out


def g4_mlp_grad(ctx, w_bf16, feat, target, tau=0.0):
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=ctx.device)
    loss = torch.empty(1, dtype=torch.float32, device=ctx.device)
    ctx.check(_L.g4_mlp_grad(ctx.h, _ptr(w_bf16), _ptr(feat), _ptr(target), feat.shape[0], float(tau), _ptr(grad),
                             _ptr(loss)))
    return grad, loss


def g4_mlp_adam(ctx, w_bf16, master, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    ctx.check(_L.g4_mlp_adam(ctx.h, _ptr(w_bf16), _ptr(master), _ptr(m), _ptr(v), _ptr(grad), float(lr),
                             float(beta1), float(beta2), float(eps), int(step)))


def g4_mlp_train_step(ctx, w_bf16, master, adam_state, grad, feat, target, lr, step, loss, tau=0.0):
    ctx.check(_L.g4_mlp_train_step(ctx.h, _ptr(w_bf16), _ptr(master), _ptr(adam_state), _ptr(grad), _ptr(feat),
                                   _ptr(target), feat.shape[0], float(tau), float(lr), int(step), _ptr(loss)))


# ------------------------------------------------------------------ FMM
def fmm_params(kernel=0, G=1.0, eps0=0.0, r_s=1.0, r_cut=1e30, theta=0.5, deterministic=0, criterion=0,
               alpha=0.005, a_seed=None, ewald=None):
    """criterion 1: the relative node-node criterion with |a| per particle
    (a_seed, float32 device tensor in caller order); ewald: the EwaldTable of
    the box for kernel 2."""
    fp = g4_fmm_params()
    fp.kernel, fp.G, fp.eps0, fp.r_s, fp.r_cut, fp.theta = int(kernel), float(G), float(eps0), float(r_s), float(r_cut), float(theta)
    fp.deterministic = int(deterministic)
    fp.criterion, fp.alpha = int(criterion), float(alpha)
    fp.a_seed = None if a_seed is None else a_seed.data_ptr()
    if ewald is not None:
        fp.ewald_table, fp.ewald_n = ewald.ptr, int(ewald.ne)
    fp._keep = (a_seed, ewald)
    return fp


def g4_fmm_workspace_bytes(tree, fp, list_factor=1.0):
    b = C.c_size_t()
    code = _L.g4_fmm_workspace_bytes(tree.h, C.byref(fp), float(list_factor), C.byref(b))
    if code != G4_OK:
        raise G4Error(code, "fmm workspace size query failed")
    return int(b.value)


def g4_fmm_force(ctx, tree, fp, list_factor=1.0, ws=None, want_pot=False, want_stats=False, out=None, retries=4):
    """FMM forces; on G4_ENOMEM (interaction lists larger than the workspace)
    the list factor grows 4x and the call is repeated."""
    ax, ay, az, pot, _, _ = out if out is not None else _force_outputs(tree.n, ctx.device, want_pot, False, False)
    st = g4_stats() if want_stats else None
    for attempt in range(retries + 1):
        nbytes = g4_fmm_workspace_bytes(tree, fp, list_factor)
        if ws is None or ws.numel() < nbytes + 256:
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
        off = (-ws.data_ptr()) % 256
        wsv = ws[off:]
        code = _L.g4_fmm_force(ctx.h, tree.h, C.byref(fp), float(list_factor), C.c_void_p(wsv.data_ptr()),
                               wsv.numel(), _ptr(ax), _ptr(ay), _ptr(az), _ptr(pot),
                               C.byref(st) if st is not None else None)
        if code == G4_ENOMEM and attempt < retries:
            list_factor *= 4.0
            continue
        ctx.check(code)
        break
    return dict(ax=ax, ay=ay, az=az, pot=pot, stats=st.as_dict() if st is not None else None, ws=ws,
                list_factor=list_factor)


def g4_fmm_force_noalloc(ctx, tree, fp, want_pot=False, want_stats=False, out=None):
    """FMM forces with the library's static device scratch (no workspace)."""
    ax, ay, az, pot, _, _ = out if out is not None else _force_outputs(tree.n, ctx.device, want_pot, False, False)
    st = g4_stats() if want_stats else None
    ctx.check(_L.g4_fmm_force_noalloc(ctx.h, tree.h, C.byref(fp), _ptr(ax), _ptr(ay), _ptr(az), _ptr(pot),
                                      C.byref(st) if st is not None else None))
    return dict(ax=ax, ay=ay, az=az, pot=pot, stats=st.as_dict() if st is not None else None)


# ------------------------------------------------------------------ forest
def g4_forest_workspace_bytes(tp, nbox, n):
    b = C.c_size_t()
    code = _L.g4_forest_workspace_bytes(C.byref(tp), int(nbox), int(n), C.byref(b))
    if code != G4_OK:
        raise G4Error(code, "forest workspace size query failed")
    return int(b.value)


def g4_build_forest(ctx, box_offsets, p, tp, ws=None):
    """box_offsets: host sequence of nbox + 1 int64 (particles grouped by box)."""
    import numpy as _np
    off = _np.ascontiguousarray(_np.asarray(box_offsets, dtype=_np.int64))
    nbox = off.shape[0] - 1
    nbytes = g4_forest_workspace_bytes(tp, nbox, p.n)
    if ws is None:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
    o = (-ws.data_ptr()) % 256
    wsv = ws[o:]
    h = C.c_void_p()
    ctx.check(_L.g4_build_forest(ctx.h, nbox, off.ctypes.data_as(C.c_void_p), C.byref(p), C.byref(tp),
                                 C.c_void_p(wsv.data_ptr()), wsv.numel(), C.byref(h)))
    t = Tree(ctx, h, ws, tp, int(p.n), p)
    t.box_offsets = off
    return t
