"""Python access to the FP64 CPU oracle -- test infrastructure only.

Loads ``oracle/liboracle.so`` (built from ``oracle.c`` by ``oracle/build.py``)
through ctypes and exposes one function per sum.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark use this module; the product
path (``paper_1909_11085_amd``) never imports it.

All arrays are NumPy float64 in structure-of-arrays layout: a 3-vector field
over N points has shape (3, N).  Group ids are int32 of shape (N,).

The sums follow the paper's single-layer potential (eq. sl_stokes), its
double-layer kernel (after eq. double_layer_int_eq), the smooth N-body
quadrature (eq. smooth_double_layer_int_eq_patches_disc) and the "other cells
only" rule of the explicit time step (Sec. 2.2, step 1(d)).  See ``oracle.c``
for the formulas.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None

EXCL_NONE = 0
EXCL_SAME_GROUP = 1
KERNEL_SL = 0
KERNEL_DL = 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from oracle.build import build as _build
        _build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_sl.argtypes = [_i64, _dp, _dp, _dp, _ip, _i64, _dp, _ip, ctypes.c_double, ctypes.c_int, _dp]
    lib.oracle_dl.argtypes = [_i64, _dp, _dp, _dp, _dp, _ip, _i64, _dp, _ip, ctypes.c_int, _dp]
    lib.oracle_p2p.argtypes = [ctypes.c_int, _i64, _dp, _dp, _dp, _dp, _ip, _i64, _dp, _ip,
                               ctypes.c_int32, _lp, _lp, _lp, _ip, ctypes.c_double, ctypes.c_int, _dp]
    lib.oracle_sl_vjp.argtypes = [_i64, _dp, _dp, _dp, _ip, _i64, _dp, _ip, ctypes.c_double,
                                  ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.oracle_dl_vjp.argtypes = [_i64, _dp, _dp, _dp, _dp, _ip, _i64, _dp, _ip, ctypes.c_int,
                                  _dp, _dp, _dp, _dp]
    for fn in ("oracle_sl", "oracle_dl", "oracle_p2p", "oracle_sl_vjp", "oracle_dl_vjp"):
        getattr(lib, fn).restype = None
    _lib = lib
    return lib


def num_threads() -> int:
    """OpenMP threads the oracle runs on (set OMP_NUM_THREADS to change)."""
    return int(_load().oracle_num_threads())


def _vec(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (3, n):
        raise ValueError(f"expected shape (3, {n}), got {a.shape}")
    return a


def _scal(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def _groups(g, n):
    if g is None:
        return np.zeros(n, dtype=np.int32)
    g = np.ascontiguousarray(g, dtype=np.int32)
    if g.shape != (n,):
        raise ValueError(f"expected group shape ({n},), got {g.shape}")
    return g


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _opt_out(shape, want):
    return np.zeros(shape, dtype=np.float64) if want else None


def _optp(a):
    return _p(a) if a is not None else None


def sl(src, f, w, trg, mu=1.0, src_group=None, trg_group=None, exclude_same_group=False):
    """Single-layer sum u(x_n) = 1/(8 pi mu) sum_m' [q/rho + r (r.q)/rho^3], q = w f."""
    ns, nt = src.shape[1], trg.shape[1]
    y, f, w, x = _vec(src, ns), _vec(f, ns), _scal(w, ns), _vec(trg, nt)
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    u = np.zeros((3, nt))
    _load().oracle_sl(ns, _p(y), _p(f), _p(w), _p(gs, _ip), nt, _p(x), _p(gt, _ip), float(mu),
                      EXCL_SAME_GROUP if exclude_same_group else EXCL_NONE, _p(u))
    return u


def dl(src, phi, w, nrm, trg, src_group=None, trg_group=None, exclude_same_group=False):
    """Double-layer sum u(x_n) = 6/(8 pi) sum_m' r (r.n_m)(r.q_m)/rho^5, q = w phi."""
    ns, nt = src.shape[1], trg.shape[1]
    y, p, w, nv, x = _vec(src, ns), _vec(phi, ns), _scal(w, ns), _vec(nrm, ns), _vec(trg, nt)
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    u = np.zeros((3, nt))
    _load().oracle_dl(ns, _p(y), _p(p), _p(w), _p(nv), _p(gs, _ip), nt, _p(x), _p(gt, _ip),
                      EXCL_SAME_GROUP if exclude_same_group else EXCL_NONE, _p(u))
    return u


def p2p(kernel, src, f, w, trg, src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, nrm=None, mu=1.0,
        src_group=None, trg_group=None, exclude_same_group=False):
    """Leaf-to-leaf sums: each target leaf sums over the sources of its interaction list."""
    ns, nt = src.shape[1], trg.shape[1]
    y, f, w, x = _vec(src, ns), _vec(f, ns), _scal(w, ns), _vec(trg, nt)
    nv = _vec(nrm, ns) if nrm is not None else np.zeros((3, ns))
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    so = np.ascontiguousarray(src_leaf_ofs, dtype=np.int64)
    to = np.ascontiguousarray(trg_leaf_ofs, dtype=np.int64)
    uo = np.ascontiguousarray(ulist_ofs, dtype=np.int64)
    ul = np.ascontiguousarray(ulist, dtype=np.int32)
    nl = len(so) - 1
    if len(to) != nl + 1 or len(uo) != nl + 1:
        raise ValueError("leaf offset arrays must all have n_leaves + 1 entries")
    u = np.zeros((3, nt))
    _load().oracle_p2p(int(kernel), ns, _p(y), _p(f), _p(w), _p(nv), _p(gs, _ip), nt, _p(x),
                       _p(gt, _ip), nl, _p(so, _lp), _p(to, _lp), _p(uo, _lp), _p(ul, _ip),
                       float(mu), EXCL_SAME_GROUP if exclude_same_group else EXCL_NONE, _p(u))
    return u


def sl_vjp(src, f, w, trg, g, mu=1.0, src_group=None, trg_group=None, exclude_same_group=False,
           want=("f", "src", "trg")):
    """Returns (dL/df, dL/dsrc, dL/dtrg) for dL/du = g; entries not in ``want`` are None."""
    ns, nt = src.shape[1], trg.shape[1]
    y, f, w, x, g = _vec(src, ns), _vec(f, ns), _scal(w, ns), _vec(trg, nt), _vec(g, nt)
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    gf, gy, gx = _opt_out((3, ns), "f" in want), _opt_out((3, ns), "src" in want), \
        _opt_out((3, nt), "trg" in want)
    _load().oracle_sl_vjp(ns, _p(y), _p(f), _p(w), _p(gs, _ip), nt, _p(x), _p(gt, _ip), float(mu),
                          EXCL_SAME_GROUP if exclude_same_group else EXCL_NONE, _p(g),
                          _optp(gf), _optp(gy), _optp(gx))
    return gf, gy, gx


def p2p_sl_vjp(src, f, w, trg, g, src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, mu=1.0, src_group=None,
               trg_group=None, exclude_same_group=False):
    """Adjoint of the single-layer leaf-to-leaf sum, (dL/df, dL/dsrc, dL/dtrg)
    for dL/du = g.  The leaf-to-leaf sum is, leaf by leaf, the direct sum from
    the concatenated sources of the leaf's list (a leaf listed k times
    contributes k times) to the leaf's targets; its adjoint is the sum over
    leaves of those direct sums' adjoints (sl_vjp), the source-side parts
    scattered back to the listed sources.  Python loop over leaves."""
    ns, nt = src.shape[1], trg.shape[1]
    y, f, w, x, g = _vec(src, ns), _vec(f, ns), _scal(w, ns), _vec(trg, nt), _vec(g, nt)
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    so, to = np.asarray(src_leaf_ofs, dtype=np.int64), np.asarray(trg_leaf_ofs, dtype=np.int64)
    uo, ul = np.asarray(ulist_ofs, dtype=np.int64), np.asarray(ulist, dtype=np.int64)
    gf, gy, gx = np.zeros((3, ns)), np.zeros((3, ns)), np.zeros((3, nt))
    for L in range(len(so) - 1):
        t = np.arange(to[L], to[L + 1])
        if t.size == 0:
            continue
        m = np.concatenate([np.arange(so[k], so[k + 1]) for k in ul[uo[L]:uo[L + 1]]] + [np.zeros(0, np.int64)])
        if m.size == 0:
            continue
        a, b, c = sl_vjp(y[:, m], f[:, m], w[m], x[:, t], g[:, t], mu=mu, src_group=gs[m], trg_group=gt[t],
                         exclude_same_group=exclude_same_group)
        for q in range(3):
            np.add.at(gf[q], m, a[q])
            np.add.at(gy[q], m, b[q])
        gx[:, t] += c
    return gf, gy, gx


def p2p_dl_vjp(src, phi, w, nrm, trg, g, src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, src_group=None,
               trg_group=None, exclude_same_group=False):
    """Adjoint of the double-layer leaf-to-leaf sum, (dL/dphi, dL/dsrc,
    dL/dtrg) for dL/du = g: as p2p_sl_vjp, leaf by leaf the adjoint (dl_vjp)
    of the direct sum from the concatenated sources of the leaf's list."""
    ns, nt = src.shape[1], trg.shape[1]
    y, p, w, nv = _vec(src, ns), _vec(phi, ns), _scal(w, ns), _vec(nrm, ns)
    x, g = _vec(trg, nt), _vec(g, nt)
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    so, to = np.asarray(src_leaf_ofs, dtype=np.int64), np.asarray(trg_leaf_ofs, dtype=np.int64)
    uo, ul = np.asarray(ulist_ofs, dtype=np.int64), np.asarray(ulist, dtype=np.int64)
    gp, gy, gx = np.zeros((3, ns)), np.zeros((3, ns)), np.zeros((3, nt))
    for L in range(len(so) - 1):
        t = np.arange(to[L], to[L + 1])
        if t.size == 0:
            continue
        m = np.concatenate([np.arange(so[k], so[k + 1]) for k in ul[uo[L]:uo[L + 1]]] + [np.zeros(0, np.int64)])
        if m.size == 0:
            continue
        a, b, c = dl_vjp(y[:, m], p[:, m], w[m], nv[:, m], x[:, t], g[:, t], src_group=gs[m], trg_group=gt[t],
                         exclude_same_group=exclude_same_group)
        for q in range(3):
            np.add.at(gp[q], m, a[q])
            np.add.at(gy[q], m, b[q])
        gx[:, t] += c
    return gp, gy, gx


def dl_vjp(src, phi, w, nrm, trg, g, src_group=None, trg_group=None, exclude_same_group=False,
           want=("phi", "src", "trg")):
    """Returns (dL/dphi, dL/dsrc, dL/dtrg) for dL/du = g; entries not in ``want`` are None."""
    ns, nt = src.shape[1], trg.shape[1]
    y, p, w, nv = _vec(src, ns), _vec(phi, ns), _scal(w, ns), _vec(nrm, ns)
    x, g = _vec(trg, nt), _vec(g, nt)
    gs, gt = _groups(src_group, ns), _groups(trg_group, nt)
    gp, gy, gx = _opt_out((3, ns), "phi" in want), _opt_out((3, ns), "src" in want), \
        _opt_out((3, nt), "trg" in want)
    _load().oracle_dl_vjp(ns, _p(y), _p(p), _p(w), _p(nv), _p(gs, _ip), nt, _p(x), _p(gt, _ip),
                          EXCL_SAME_GROUP if exclude_same_group else EXCL_NONE, _p(g),
                          _optp(gp), _optp(gy), _optp(gx))
    return gp, gy, gx
