"""PyTorch-facing API of the MI355X Stokes kernel-sum library.

Thin marshalling over the C ABI: tensors supply device pointers, torch's
current stream supplies the HIP stream and torch's caching allocator supplies
the workspace.  All arithmetic runs in the HIP kernels; there is no CPU or
PyTorch fallback.

Layout: 3-vector fields are float64 tensors of shape (3, N), contiguous, on
the GPU; weights (N,) float64; group ids (N,) int32.
"""
from __future__ import annotations

import ctypes
import threading

import numpy as np
import torch

from . import _capi as C

_ctx_lock = threading.Lock()
_ctxs = {}

PRECISIONS = {"fp64": C.FP64, "mixed": C.MIXED}


def context(device=None):
    """The library context of a CUDA/HIP device (created once per device)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    with _ctx_lock:
        if idx not in _ctxs:
            h = ctypes.c_void_p()
            C.check(C.lib().stokes_create(ctypes.byref(h), idx))
            _ctxs[idx] = h
        return _ctxs[idx]


def set_grid_override(workgroups, device=None):
    """Force the workgroup count of direct sums (0 = the resident count)."""
    C.check(C.lib().stokes_set_grid_override(context(device), int(workgroups)))


def set_pair_symmetry(on=True, device=None):
    """Evaluate each unordered pair once on shared point sets (default on)."""
    C.check(C.lib().stokes_set_pair_symmetry(context(device), int(bool(on))))


def debug_pair_classes(classes, device=None):
    """Test-only: register an int32 (n_trg, n_src) device tensor (zeroed) that
    the mixed direct and leaf-to-leaf sums of those sizes fill with the class
    code of every pair they take (see stokes_debug_pair_classes); None
    unregisters."""
    if classes is None:
        C.check(C.lib().stokes_debug_pair_classes(context(device), None, 0, 0))
        return
    if classes.dtype != torch.int32 or classes.dim() != 2 or not classes.is_contiguous():
        raise ValueError("classes must be a contiguous int32 (n_trg, n_src) tensor")
    C.check(C.lib().stokes_debug_pair_classes(context(classes.device), _ptr(classes), classes.shape[0],
                                              classes.shape[1]))


def timing_enable(on=True, device=None):
    """Record HIP events around each evaluation's main summation kernel."""
    C.check(C.lib().stokes_timing_enable(context(device), int(bool(on))))


def timing_read(device=None):
    """(summed milliseconds, launches) of the main kernels timed since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    C.check(C.lib().stokes_timing_read(context(device), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _vec3(t, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dim() != 2 or t.shape[0] != 3:
        raise ValueError(f"{name} must have shape (3, N), got {tuple(t.shape)}")
    if t.dtype != torch.float64 or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on {device}")
    return t


def _vec1(t, n, name, device, dtype=torch.float64):
    if t.shape != (n,) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape ({n},) on {device}")
    return t


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class _Rule:
    """Keeps the tensors of a stokes_exclusion alive for the duration of a call."""

    def __init__(self, device, n_src, n_trg, src_group, trg_group, exclude_same_group, precision,
                 group_h, near_frac):
        if exclude_same_group is None:
            exclude_same_group = src_group is not None and trg_group is not None
        self.tensors = []
        sg = tg = gh = None
        if src_group is not None:
            sg = _vec1(src_group, n_src, "src_group", device, torch.int32)
        if trg_group is not None:
            tg = _vec1(trg_group, n_trg, "trg_group", device, torch.int32)
        if exclude_same_group and (sg is None or tg is None):
            raise ValueError("exclude_same_group needs src_group and trg_group")
        if group_h is not None:
            gh = group_h
            if gh.dim() != 1 or gh.dtype != torch.float64 or gh.device != device or not gh.is_contiguous():
                raise ValueError("group_h must be a contiguous 1-D float64 tensor on the device")
        self.tensors = [sg, tg, gh]
        self.ex = C.Exclusion(C.EXCL_SAME_GROUP if exclude_same_group else C.EXCL_NONE,
                              _ptr(sg).value, _ptr(tg).value, _ptr(gh).value,
                              0 if gh is None else gh.numel(), float(near_frac))
        self.opts = C.Opts(PRECISIONS[precision], 0)


def _workspace(op, n_src, n_trg, n_leaves, opts, device, n_ulist=0):
    size = ctypes.c_size_t()
    C.check(C.lib().stokes_workspace_size(context(device), op, n_src, n_trg, n_leaves, n_ulist,
                                          ctypes.byref(opts), ctypes.byref(size)))
    ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=device)
    return ws, int(size.value)


def _out(out, n_trg, device, accumulate):
    if out is None:
        if accumulate:
            raise ValueError("accumulate=True needs an out tensor")
        return torch.empty((3, n_trg), dtype=torch.float64, device=device)
    return _vec3(out, "out", device)


def sl(src, f, w, trg, mu=1.0, src_group=None, trg_group=None, exclude_same_group=None,
       precision="fp64", group_h=None, near_frac=0.5, out=None, accumulate=False):
    """Single-layer (Stokeslet) sum at the targets; see stokes_sl_eval.

    Returns ``out`` (allocated if None), shape (3, n_trg)."""
    device = src.device
    _vec3(src, "src", device); _vec3(f, "f", device); _vec3(trg, "trg", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    if f.shape[1] != ns:
        raise ValueError("f must have the same number of points as src")
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, precision, group_h, near_frac)
    rule.opts.accumulate = int(bool(accumulate))
    out = _out(out, nt, device, accumulate)
    ws, size = _workspace(C.OP_SL, ns, nt, 0, rule.opts, device)
    C.check(C.lib().stokes_sl_eval(context(device), ns, _ptr(src), _ptr(f), _ptr(w), nt, _ptr(trg),
                                   float(mu), ctypes.byref(rule.ex), ctypes.byref(rule.opts),
                                   _ptr(out), _ptr(ws), size, _stream(device)))
    return out


def dl(src, phi, w, nrm, trg, src_group=None, trg_group=None, exclude_same_group=None,
       precision="fp64", group_h=None, near_frac=0.5, out=None, accumulate=False):
    """Double-layer (stresslet) sum at the targets; see stokes_dl_eval."""
    device = src.device
    _vec3(src, "src", device); _vec3(phi, "phi", device); _vec3(nrm, "nrm", device)
    _vec3(trg, "trg", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    if phi.shape[1] != ns or nrm.shape[1] != ns:
        raise ValueError("phi and nrm must have the same number of points as src")
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, precision, group_h, near_frac)
    rule.opts.accumulate = int(bool(accumulate))
    out = _out(out, nt, device, accumulate)
    ws, size = _workspace(C.OP_DL, ns, nt, 0, rule.opts, device)
    C.check(C.lib().stokes_dl_eval(context(device), ns, _ptr(src), _ptr(phi), _ptr(w), _ptr(nrm),
                                   nt, _ptr(trg), ctypes.byref(rule.ex), ctypes.byref(rule.opts),
                                   _ptr(out), _ptr(ws), size, _stream(device)))
    return out


# ----------------------------------------------------------------------------
# adjoints
# ----------------------------------------------------------------------------
def _grad_out(t, n, name, device):
    if t is None:
        return None
    return _vec3(t, name, device)


def sl_vjp(src, f, w, trg, grad_u, mu=1.0, src_group=None, trg_group=None, exclude_same_group=None,
           grad_f=None, grad_src=None, grad_trg=None, accumulate=False):
    """Vector-Jacobian product of the single-layer sum (see stokes_sl_vjp).

    Writes into the given (3, N) float64 tensors; any may be None.  For a
    shared point set (src is trg) grad_src and grad_trg may be the same tensor,
    which then receives the total position gradient from one fused pass."""
    device = src.device
    _vec3(src, "src", device); _vec3(f, "f", device); _vec3(trg, "trg", device)
    _vec3(grad_u, "grad_u", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, "fp64", None, 0.0)
    rule.opts.accumulate = int(bool(accumulate))
    gf, gs, gt = (_grad_out(grad_f, ns, "grad_f", device), _grad_out(grad_src, ns, "grad_src", device),
                  _grad_out(grad_trg, nt, "grad_trg", device))
    ws, size = _workspace(C.OP_SL_VJP, ns, nt, 0, rule.opts, device)
    C.check(C.lib().stokes_sl_vjp(context(device), ns, _ptr(src), _ptr(f), _ptr(w), nt, _ptr(trg),
                                  float(mu), ctypes.byref(rule.ex), ctypes.byref(rule.opts),
                                  _ptr(grad_u), _ptr(gf), _ptr(gs), _ptr(gt), _ptr(ws), size,
                                  _stream(device)))
    return gf, gs, gt


def dl_vjp(src, phi, w, nrm, trg, grad_u, src_group=None, trg_group=None, exclude_same_group=None,
           grad_phi=None, grad_src=None, grad_trg=None, accumulate=False):
    """Vector-Jacobian product of the double-layer sum (see stokes_dl_vjp)."""
    device = src.device
    _vec3(src, "src", device); _vec3(phi, "phi", device); _vec3(nrm, "nrm", device)
    _vec3(trg, "trg", device); _vec3(grad_u, "grad_u", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, "fp64", None, 0.0)
    rule.opts.accumulate = int(bool(accumulate))
    gp, gs, gt = (_grad_out(grad_phi, ns, "grad_phi", device), _grad_out(grad_src, ns, "grad_src", device),
                  _grad_out(grad_trg, nt, "grad_trg", device))
    ws, size = _workspace(C.OP_DL_VJP, ns, nt, 0, rule.opts, device)
    C.check(C.lib().stokes_dl_vjp(context(device), ns, _ptr(src), _ptr(phi), _ptr(w), _ptr(nrm), nt,
                                  _ptr(trg), ctypes.byref(rule.ex), ctypes.byref(rule.opts),
                                  _ptr(grad_u), _ptr(gp), _ptr(gs), _ptr(gt), _ptr(ws), size,
                                  _stream(device)))
    return gp, gs, gt


def _empty3(n, like):
    return torch.empty((3, n), dtype=torch.float64, device=like.device)


class StokesSL(torch.autograd.Function):
    """Single-layer sum differentiable in the density and in both point sets
    (weights are constants).  The backward runs the float64 adjoint."""

    @staticmethod
    def forward(ctx, src, f, w, trg, mu, src_group, trg_group, exclude_same_group, precision, group_h,
                near_frac):
        u = sl(src, f, w, trg, mu=mu, src_group=src_group, trg_group=trg_group,
               exclude_same_group=exclude_same_group, precision=precision, group_h=group_h,
               near_frac=near_frac)
        ctx.save_for_backward(src, f, w, trg)
        ctx.args = (mu, src_group, trg_group, exclude_same_group)
        ctx.shared = src is trg
        return u

    @staticmethod
    def backward(ctx, grad_u):
        src, f, w, trg = ctx.saved_tensors
        mu, sg, tg, ex = ctx.args
        need_f, need_src, need_trg = ctx.needs_input_grad[1], ctx.needs_input_grad[0], ctx.needs_input_grad[3]
        grad_u = grad_u.contiguous()
        gf = _empty3(src.shape[1], src) if need_f else None
        if ctx.shared and (need_src or need_trg):
            gpos = _empty3(src.shape[1], src)
            sl_vjp(src, f, w, trg, grad_u, mu=mu, src_group=sg, trg_group=tg, exclude_same_group=ex,
                   grad_f=gf, grad_src=gpos, grad_trg=gpos)
            return gpos, gf, None, None, None, None, None, None, None, None, None
        gs = _empty3(src.shape[1], src) if need_src else None
        gt = _empty3(trg.shape[1], trg) if need_trg else None
        if gf is not None or gs is not None or gt is not None:
            sl_vjp(src, f, w, trg, grad_u, mu=mu, src_group=sg, trg_group=tg, exclude_same_group=ex,
                   grad_f=gf, grad_src=gs, grad_trg=gt)
        return gs, gf, None, gt, None, None, None, None, None, None, None


class StokesDL(torch.autograd.Function):
    """Double-layer sum differentiable in the density and in both point sets
    (weights and normals are constants).  Float64 adjoint."""

    @staticmethod
    def forward(ctx, src, phi, w, nrm, trg, src_group, trg_group, exclude_same_group, precision,
                group_h, near_frac):
        u = dl(src, phi, w, nrm, trg, src_group=src_group, trg_group=trg_group,
               exclude_same_group=exclude_same_group, precision=precision, group_h=group_h,
               near_frac=near_frac)
        ctx.save_for_backward(src, phi, w, nrm, trg)
        ctx.args = (src_group, trg_group, exclude_same_group)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        src, phi, w, nrm, trg = ctx.saved_tensors
        sg, tg, ex = ctx.args
        need_src, need_phi, need_trg = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[4]
        grad_u = grad_u.contiguous()
        gp = _empty3(src.shape[1], src) if need_phi else None
        gs = _empty3(src.shape[1], src) if need_src else None
        gt = _empty3(trg.shape[1], trg) if need_trg else None
        if gp is not None or gs is not None or gt is not None:
            dl_vjp(src, phi, w, nrm, trg, grad_u, src_group=sg, trg_group=tg, exclude_same_group=ex,
                   grad_phi=gp, grad_src=gs, grad_trg=gt)
        return gs, gp, None, None, gt, None, None, None, None, None, None


def sl_diff(src, f, w, trg, mu=1.0, src_group=None, trg_group=None, exclude_same_group=None,
            precision="fp64", group_h=None, near_frac=0.5):
    """Differentiable single-layer sum (torch.autograd)."""
    return StokesSL.apply(src, f, w, trg, mu, src_group, trg_group, exclude_same_group, precision,
                          group_h, near_frac)


def dl_diff(src, phi, w, nrm, trg, src_group=None, trg_group=None, exclude_same_group=None,
            precision="fp64", group_h=None, near_frac=0.5):
    """Differentiable double-layer sum (torch.autograd)."""
    return StokesDL.apply(src, phi, w, nrm, trg, src_group, trg_group, exclude_same_group, precision,
                          group_h, near_frac)


# ----------------------------------------------------------------------------
# leaf-to-leaf (P2P) sums
# ----------------------------------------------------------------------------
class P2PPlan:
    """Leaf layout on the device (see stokes_p2p_plan_create).

    Host NumPy arrays: src_leaf_ofs, trg_leaf_ofs, ulist_ofs (int64,
    n_leaves + 1 entries) and ulist (int32).  Points are in leaf order."""

    def __init__(self, src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, n_src, n_trg, device=None):
        import numpy as np
        self._so = np.ascontiguousarray(src_leaf_ofs, dtype=np.int64)
        self._to = np.ascontiguousarray(trg_leaf_ofs, dtype=np.int64)
        self._uo = np.ascontiguousarray(ulist_ofs, dtype=np.int64)
        self._ul = np.ascontiguousarray(ulist, dtype=np.int32)
        self.n_leaves = len(self._so) - 1
        if len(self._to) != self.n_leaves + 1 or len(self._uo) != self.n_leaves + 1:
            raise ValueError("leaf offset arrays must all have n_leaves + 1 entries")
        self.n_src, self.n_trg = int(n_src), int(n_trg)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._lib = C.lib()
        h = ctypes.c_void_p()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        C.check(self._lib.stokes_p2p_plan_create(context(self.device), self.n_leaves, self.n_src, self.n_trg,
                                                 vp(self._so), vp(self._to), vp(self._uo), vp(self._ul),
                                                 len(self._ul), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def device_arrays(self):
        """The layout as device tensors (src_leaf_ofs, trg_leaf_ofs, ulist_ofs,
        ulist), uploaded on first use and kept."""
        if getattr(self, "_dev", None) is None:
            self._dev = tuple(torch.from_numpy(a).to(self.device) for a in (self._so, self._to, self._uo, self._ul))
        return self._dev

    def pairs(self):
        """Pairs visited (before the pair rule removes any)."""
        n = ctypes.c_int64()
        C.check(self._lib.stokes_p2p_plan_pairs(self._h, ctypes.byref(n)))
        return n.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.stokes_p2p_plan_destroy(h)
            self._h = None


def _device_layout(layout, device):
    """(src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, n_leaves) as device
    tensors, from a P2PPlan or a tuple of four device tensors."""
    if isinstance(layout, P2PPlan):
        if layout.device != device:
            raise ValueError("the plan lives on another device than the points")
        so, to, uo, ul = layout.device_arrays()
    else:
        so, to, uo, ul = layout
    for t, name, dt in ((so, "src_leaf_ofs", torch.int64), (to, "trg_leaf_ofs", torch.int64),
                        (uo, "ulist_ofs", torch.int64), (ul, "ulist", torch.int32)):
        if t.dtype != dt or t.dim() != 1 or t.device != device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous 1-D {dt} tensor on the points' device")
    n_leaves = so.numel() - 1
    if n_leaves < 0 or to.numel() != n_leaves + 1 or uo.numel() != n_leaves + 1:
        raise ValueError("the leaf offset arrays must all have n_leaves + 1 entries")
    return so, to, uo, ul, n_leaves


def p2p_leaf(layout, src, f, w, trg, kernel="sl", nrm=None, mu=1.0, src_group=None, trg_group=None,
             exclude_same_group=None, precision="fp64", group_h=None, near_frac=0.5, out=None,
             accumulate=False):
    """Leaf-to-leaf sum over interaction lists.

    layout: a P2PPlan (host arrays, prepared once; stokes_p2p_plan_eval), or
    the device arrays (src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist) as int64,
    int64, int64 and int32 tensors on the points' device, checked and cut into
    work items on the device at every call (stokes_p2p_leaf_eval; a malformed
    layout gives NaN outputs)."""
    device = src.device
    _vec3(src, "src", device); _vec3(f, "f", device); _vec3(trg, "trg", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    k = {"sl": C.KERNEL_SL, "dl": C.KERNEL_DL}[kernel]
    if k == C.KERNEL_DL:
        _vec3(nrm, "nrm", device)
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, precision, group_h, near_frac)
    rule.opts.accumulate = int(bool(accumulate))
    out = _out(out, nt, device, accumulate)
    op = C.OP_P2P_SL if k == C.KERNEL_SL else C.OP_P2P_DL
    nrm_p = _ptr(nrm) if k == C.KERNEL_DL else ctypes.c_void_p(0)
    if isinstance(layout, P2PPlan):
        ws, size = _workspace(op, ns, nt, layout.n_leaves, rule.opts, device)
        C.check(C.lib().stokes_p2p_plan_eval(context(device), layout.handle, k, ns, _ptr(src), _ptr(f), _ptr(w),
                                             nrm_p, nt, _ptr(trg), float(mu), ctypes.byref(rule.ex),
                                             ctypes.byref(rule.opts), _ptr(out), _ptr(ws), size, _stream(device)))
        return out
    so, to, uo, ul, n_leaves = _device_layout(layout, device)
    ws, size = _workspace(op, ns, nt, n_leaves, rule.opts, device)
    C.check(C.lib().stokes_p2p_leaf_eval(context(device), k, ns, _ptr(src), _ptr(f), _ptr(w), nrm_p, nt, _ptr(trg),
                                         n_leaves, _ptr(so), _ptr(to), _ptr(uo), _ptr(ul), ul.numel(), float(mu),
                                         ctypes.byref(rule.ex), ctypes.byref(rule.opts), _ptr(out), _ptr(ws), size,
                                         _stream(device)))
    return out


def p2p_sl_vjp(layout, src, f, w, trg, grad_u, mu=1.0, src_group=None, trg_group=None, exclude_same_group=None,
               grad_f=None, grad_src=None, grad_trg=None, accumulate=False):
    """Vector-Jacobian product of the single-layer leaf-to-leaf sum (see
    stokes_p2p_sl_vjp): the adjoint sums over the pairs the lists name.

    layout as for p2p_leaf (a P2PPlan's arrays are used on the device).  Writes
    into the given (3, N) float64 tensors; any may be None, none may overlap."""
    device = src.device
    _vec3(src, "src", device); _vec3(f, "f", device); _vec3(trg, "trg", device)
    _vec3(grad_u, "grad_u", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    if f.shape[1] != ns or grad_u.shape[1] != nt:
        raise ValueError("f must match src and grad_u must match trg")
    so, to, uo, ul, n_leaves = _device_layout(layout, device)
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, "fp64", None, 0.0)
    rule.opts.accumulate = int(bool(accumulate))
    gf, gs, gt = (_grad_out(grad_f, ns, "grad_f", device), _grad_out(grad_src, ns, "grad_src", device),
                  _grad_out(grad_trg, nt, "grad_trg", device))
    ws, size = _workspace(C.OP_P2P_SL_VJP, ns, nt, n_leaves, rule.opts, device, n_ulist=ul.numel())
    C.check(C.lib().stokes_p2p_sl_vjp(context(device), ns, _ptr(src), _ptr(f), _ptr(w), nt, _ptr(trg), n_leaves,
                                      _ptr(so), _ptr(to), _ptr(uo), _ptr(ul), ul.numel(), float(mu),
                                      ctypes.byref(rule.ex), ctypes.byref(rule.opts), _ptr(grad_u), _ptr(gf),
                                      _ptr(gs), _ptr(gt), _ptr(ws), size, _stream(device)))
    return gf, gs, gt


def p2p_dl_vjp(layout, src, phi, w, nrm, trg, grad_u, src_group=None, trg_group=None, exclude_same_group=None,
               grad_phi=None, grad_src=None, grad_trg=None, accumulate=False):
    """Vector-Jacobian product of the double-layer leaf-to-leaf sum (see
    stokes_p2p_dl_vjp); arguments as p2p_sl_vjp, plus the source normals."""
    device = src.device
    _vec3(src, "src", device); _vec3(phi, "phi", device); _vec3(nrm, "nrm", device); _vec3(trg, "trg", device)
    _vec3(grad_u, "grad_u", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    if phi.shape[1] != ns or nrm.shape[1] != ns or grad_u.shape[1] != nt:
        raise ValueError("phi and nrm must match src and grad_u must match trg")
    so, to, uo, ul, n_leaves = _device_layout(layout, device)
    rule = _Rule(device, ns, nt, src_group, trg_group, exclude_same_group, "fp64", None, 0.0)
    rule.opts.accumulate = int(bool(accumulate))
    gp, gs, gt = (_grad_out(grad_phi, ns, "grad_phi", device), _grad_out(grad_src, ns, "grad_src", device),
                  _grad_out(grad_trg, nt, "grad_trg", device))
    ws, size = _workspace(C.OP_P2P_DL_VJP, ns, nt, n_leaves, rule.opts, device, n_ulist=ul.numel())
    C.check(C.lib().stokes_p2p_dl_vjp(context(device), ns, _ptr(src), _ptr(phi), _ptr(w), _ptr(nrm), nt, _ptr(trg),
                                      n_leaves, _ptr(so), _ptr(to), _ptr(uo), _ptr(ul), ul.numel(),
                                      ctypes.byref(rule.ex), ctypes.byref(rule.opts), _ptr(grad_u), _ptr(gp),
                                      _ptr(gs), _ptr(gt), _ptr(ws), size, _stream(device)))
    return gp, gs, gt


class StokesP2P(torch.autograd.Function):
    """Leaf-to-leaf sum (single or double layer) differentiable in the density
    and in both point sets (weights and normals are constants).  The backward
    runs the float64 adjoint over the same lists; on a shared point set
    autograd adds the source-side and target-side position gradients."""

    @staticmethod
    def forward(ctx, layout, src, f, w, trg, kernel, nrm, mu, src_group, trg_group, exclude_same_group, precision,
                group_h, near_frac):
        u = p2p_leaf(layout, src, f, w, trg, kernel=kernel, nrm=nrm, mu=mu, src_group=src_group,
                     trg_group=trg_group, exclude_same_group=exclude_same_group, precision=precision,
                     group_h=group_h, near_frac=near_frac)
        ctx.save_for_backward(src, f, w, trg, nrm)
        ctx.layout = layout
        ctx.args = (kernel, mu, src_group, trg_group, exclude_same_group)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        src, f, w, trg, nrm = ctx.saved_tensors
        kernel, mu, sg, tg, ex = ctx.args
        need_src, need_f, need_trg = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[4]
        grad_u = grad_u.contiguous()
        gf = _empty3(src.shape[1], src) if need_f else None
        gs = _empty3(src.shape[1], src) if need_src else None
        gt = _empty3(trg.shape[1], trg) if need_trg else None
        if gf is not None or gs is not None or gt is not None:
            if kernel == "sl":
                p2p_sl_vjp(ctx.layout, src, f, w, trg, grad_u, mu=mu, src_group=sg, trg_group=tg,
                           exclude_same_group=ex, grad_f=gf, grad_src=gs, grad_trg=gt)
            else:
                p2p_dl_vjp(ctx.layout, src, f, w, nrm, trg, grad_u, src_group=sg, trg_group=tg,
                           exclude_same_group=ex, grad_phi=gf, grad_src=gs, grad_trg=gt)
        return None, gs, gf, None, gt, None, None, None, None, None, None, None, None, None


def p2p_diff(layout, src, f, w, trg, kernel="sl", nrm=None, mu=1.0, src_group=None, trg_group=None,
             exclude_same_group=None, precision="fp64", group_h=None, near_frac=0.5):
    """Differentiable leaf-to-leaf sum (torch.autograd), single layer (f is the
    density) or double layer (f is phi, nrm the source normals)."""
    if kernel not in ("sl", "dl"):
        raise ValueError("kernel must be 'sl' or 'dl'")
    if kernel == "dl" and nrm is None:
        raise ValueError("the double layer needs nrm")
    return StokesP2P.apply(layout, src, f, w, trg, kernel, nrm, mu, src_group, trg_group, exclude_same_group,
                           precision, group_h, near_frac)


# ----------------------------------------------------------------------------
# check-point quadrature on and near a patched surface
# ----------------------------------------------------------------------------
class _PatchRule:
    """Keeps the host node / weight arrays of a stokes_patch_rule alive."""

    def __init__(self, nodes_1d, weights_1d, eta, p=8, R_frac=0.15, r_frac=0.15):
        self.t = np.ascontiguousarray(nodes_1d, dtype=np.float64)
        self.w = np.ascontiguousarray(weights_1d, dtype=np.float64)
        if self.t.ndim != 1 or self.t.shape != self.w.shape:
            raise ValueError("nodes_1d and weights_1d must be 1-D arrays of the same length")
        dp = ctypes.POINTER(ctypes.c_double)
        self.rule = C.PatchRule(len(self.t), int(eta), int(p), float(R_frac), float(r_frac),
                                self.t.ctypes.data_as(dp), self.w.ctypes.data_as(dp))
        self.q = len(self.t)


def patch_upsample(node_xyz, nodes_1d, weights_1d, eta, density=None):
    """Fine discretisation of a patched surface; see stokes_patch_upsample.

    node_xyz (3, n_patches*q*q) and density (same shape, optional).  Returns
    (fine_xyz, fine_density or None, fine_weight, fine_normal, patch_size)."""
    device = node_xyz.device
    _vec3(node_xyz, "node_xyz", device)
    R = _PatchRule(nodes_1d, weights_1d, eta)
    qq = R.q * R.q
    if node_xyz.shape[1] % qq:
        raise ValueError("node_xyz must hold n_patches * q * q points")
    npatch = node_xyz.shape[1] // qq
    nf = npatch * (2 ** int(eta) * R.q) ** 2
    if density is not None:
        _vec3(density, "density", device)
        if density.shape != node_xyz.shape:
            raise ValueError("density must have the shape of node_xyz")
    fx = torch.empty((3, nf), dtype=torch.float64, device=device)
    fphi = torch.empty((3, nf), dtype=torch.float64, device=device) if density is not None else None
    fw = torch.empty(nf, dtype=torch.float64, device=device)
    fn = torch.empty((3, nf), dtype=torch.float64, device=device)
    L = torch.empty(npatch, dtype=torch.float64, device=device)
    C.check(C.lib().stokes_patch_upsample(context(device), npatch, ctypes.byref(R.rule), _ptr(node_xyz),
                                          _ptr(density), _ptr(fx), _ptr(fphi), _ptr(fw), _ptr(fn), _ptr(L),
                                          _stream(device)))
    return fx, fphi, fw, fn, L


def dl_checkpoint(node_xyz, density, nodes_1d, weights_1d, eta=1, p=8, R_frac=0.15, r_frac=0.15,
                  trg_patch=None, trg_uvd=None, precision="fp64", out=None, accumulate=False,
                  return_check=False):
    """Double-layer velocity on or near a patched surface by the check-point
    quadrature; see stokes_dl_checkpoint_eval.

    Targets: every node on the surface (trg_patch = trg_uvd = None), or
    trg_patch (M,) int32 with trg_uvd (3, M) rows u, v, d.  Returns vel (3, M);
    with return_check also the check points and their velocities, each
    (3, M*(p+1))."""
    device = node_xyz.device
    _vec3(node_xyz, "node_xyz", device)
    _vec3(density, "density", device)
    if density.shape != node_xyz.shape:
        raise ValueError("density must have the shape of node_xyz")
    R = _PatchRule(nodes_1d, weights_1d, eta, p, R_frac, r_frac)
    qq = R.q * R.q
    if node_xyz.shape[1] % qq:
        raise ValueError("node_xyz must hold n_patches * q * q points")
    npatch = node_xyz.shape[1] // qq
    if (trg_patch is None) != (trg_uvd is None):
        raise ValueError("trg_patch and trg_uvd go together")
    if trg_patch is None:
        m = node_xyz.shape[1]
    else:
        m = trg_patch.shape[0]
        _vec1(trg_patch, m, "trg_patch", device, torch.int32)
        _vec3(trg_uvd, "trg_uvd", device)
        if trg_uvd.shape[1] != m:
            raise ValueError("trg_uvd must have shape (3, len(trg_patch))")
    opts = C.Opts(PRECISIONS[precision], int(bool(accumulate)))
    out = _out(out, m, device, accumulate)
    cx = cv = None
    if return_check:
        cx = torch.empty((3, m * (p + 1)), dtype=torch.float64, device=device)
        cv = torch.empty((3, m * (p + 1)), dtype=torch.float64, device=device)
    size = ctypes.c_size_t()
    C.check(C.lib().stokes_checkpoint_workspace_size(context(device), npatch, ctypes.byref(R.rule), m,
                                                     ctypes.byref(opts), ctypes.byref(size)))
    ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=device)
    C.check(C.lib().stokes_dl_checkpoint_eval(context(device), npatch, ctypes.byref(R.rule), _ptr(node_xyz),
                                              _ptr(density), m, _ptr(trg_patch), _ptr(trg_uvd),
                                              ctypes.byref(opts), _ptr(out), _ptr(cx), _ptr(cv), _ptr(ws),
                                              int(size.value), _stream(device)))
    return (out, cx, cv) if return_check else out


def _bie_common(node_xyz, nodes_1d, weights_1d, eta, p, R_frac, r_frac, max_iter, precision, accumulate=False):
    device = node_xyz.device
    _vec3(node_xyz, "node_xyz", device)
    R = _PatchRule(nodes_1d, weights_1d, eta, p, R_frac, r_frac)
    qq = R.q * R.q
    if node_xyz.shape[1] % qq:
        raise ValueError("node_xyz must hold n_patches * q * q points")
    opts = C.Opts(PRECISIONS[precision], int(bool(accumulate)))
    size = ctypes.c_size_t()
    npatch = node_xyz.shape[1] // qq
    C.check(C.lib().stokes_bie_workspace_size(context(device), npatch, ctypes.byref(R.rule), int(max_iter),
                                              ctypes.byref(opts), ctypes.byref(size)))
    ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=device)
    return device, R, npatch, opts, ws, int(size.value)


def bie_apply(node_xyz, phi, nodes_1d, weights_1d, eta=1, p=8, R_frac=0.15, r_frac=0.15, precision="fp64",
              out=None, accumulate=False):
    """(L_in - N) phi at the nodes of a closed patched surface; see stokes_bie_apply."""
    device, R, npatch, opts, ws, size = _bie_common(node_xyz, nodes_1d, weights_1d, eta, p, R_frac, r_frac, 0,
                                                    precision, accumulate)
    _vec3(phi, "phi", device)
    if phi.shape != node_xyz.shape:
        raise ValueError("phi must have the shape of node_xyz")
    out = _out(out, node_xyz.shape[1], device, accumulate)
    C.check(C.lib().stokes_bie_apply(context(device), npatch, ctypes.byref(R.rule), _ptr(node_xyz), _ptr(phi),
                                     ctypes.byref(opts), _ptr(out), _ptr(ws), size, _stream(device)))
    return out


def bie_solve(node_xyz, g, nodes_1d, weights_1d, eta=1, p=8, R_frac=0.15, r_frac=0.15, max_iter=30, rtol=1e-10,
              precision="fp64", out=None):
    """GMRES on (L_in - N) phi = g; see stokes_bie_solve.  Returns (phi,
    iterations, residual history as a NumPy array of iterations + 1 entries)."""
    device, R, npatch, opts, ws, size = _bie_common(node_xyz, nodes_1d, weights_1d, eta, p, R_frac, r_frac,
                                                    max_iter, precision)
    _vec3(g, "g", device)
    if g.shape != node_xyz.shape:
        raise ValueError("g must have the shape of node_xyz")
    out = _out(out, node_xyz.shape[1], device, False)
    its = ctypes.c_int32()
    hist = (ctypes.c_double * (int(max_iter) + 1))()
    C.check(C.lib().stokes_bie_solve(context(device), npatch, ctypes.byref(R.rule), _ptr(node_xyz), _ptr(g),
                                     int(max_iter), float(rtol), ctypes.byref(opts), _ptr(out), ctypes.byref(its),
                                     hist, _ptr(ws), size, _stream(device)))
    return out, its.value, np.array(hist[: its.value + 1])


# ----------------------------------------------------------------------------
# collision candidates by spatial hashing
# ----------------------------------------------------------------------------
def space_time_boxes(mesh_ofs, x0, x1=None, inflate=0.0):
    """Space-time bounding box per mesh; see stokes_space_time_boxes.

    mesh_ofs: int64 tensor (n_meshes + 1,) on the device.  Returns (lo, hi),
    each (3, n_meshes)."""
    device = x0.device
    _vec3(x0, "x0", device)
    if x1 is not None:
        _vec3(x1, "x1", device)
        if x1.shape != x0.shape:
            raise ValueError("x1 must have the shape of x0")
    nm = mesh_ofs.numel() - 1
    _vec1(mesh_ofs, nm + 1, "mesh_ofs", device, torch.int64)
    lo = torch.empty((3, nm), dtype=torch.float64, device=device)
    hi = torch.empty((3, nm), dtype=torch.float64, device=device)
    C.check(C.lib().stokes_space_time_boxes(context(device), nm, _ptr(mesh_ofs), x0.shape[1], _ptr(x0), _ptr(x1),
                                            float(inflate), _ptr(lo), _ptr(hi), _stream(device)))
    return lo, hi


def collision_candidates(lo, hi, cell_size, max_entries=None, capacity=None):
    """Pairs of boxes sharing a grid cell; see stokes_collision_candidates.

    Returns an int32 tensor (2, n_pairs) on the device.  max_entries defaults
    to 64 per box; capacity to what a first counting call reports."""
    device = lo.device
    _vec3(lo, "lo", device)
    _vec3(hi, "hi", device)
    nb = lo.shape[1]
    if hi.shape != lo.shape:
        raise ValueError("hi must have the shape of lo")
    max_entries = 64 * max(nb, 1) if max_entries is None else int(max_entries)
    size = ctypes.c_size_t()
    C.check(C.lib().stokes_collision_workspace_size(context(device), nb, max_entries, ctypes.byref(size)))
    ws = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=device)
    n_pairs, n_entries = ctypes.c_int64(), ctypes.c_int64()

    def call(buf, cap):
        C.check(C.lib().stokes_collision_candidates(context(device), nb, _ptr(lo), _ptr(hi), float(cell_size),
                                                    max_entries, _ptr(buf), cap, ctypes.byref(n_pairs),
                                                    ctypes.byref(n_entries), _ptr(ws), int(size.value),
                                                    _stream(device)))

    if capacity is None:
        call(None, 0)
        capacity = n_pairs.value
    out = torch.empty((2, max(int(capacity), 1)), dtype=torch.int32, device=device)
    call(out, int(capacity))
    return out[:, : min(n_pairs.value, int(capacity))]


# ----------------------------------------------------------------------------
# fast multipole method (single layer)
# ----------------------------------------------------------------------------
class FMMPlan:
    """Check-to-equivalent operators of one surface order, on the device; see
    stokes_fmm_plan_create."""

    def __init__(self, order=4, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._h = ctypes.c_void_p()
        C.check(C.lib().stokes_fmm_plan_create(context(self.device), int(order), ctypes.byref(self._h)))
        self.order = int(order)

    @property
    def handle(self):
        return self._h

    def device_arrays(self):
        """The layout as device tensors (src_leaf_ofs, trg_leaf_ofs, ulist_ofs,
        ulist), uploaded on first use and kept."""
        if getattr(self, "_dev", None) is None:
            self._dev = tuple(torch.from_numpy(a).to(self.device) for a in (self._so, self._to, self._uo, self._ul))
        return self._dev

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        try:
            if h is not None and h.value:
                C.lib().stokes_fmm_plan_destroy(h)
        except Exception:                 # interpreter shutdown: the library may be gone
            pass


def _fmm_precision(precision):
    if precision not in ("fp64", "mixed"):
        raise ValueError("precision must be 'fp64' or 'mixed'")
    return C.MIXED if precision == "mixed" else C.FP64


class _FmmRule:
    """Keeps the tensors of the FMM's pair rule alive for a call."""

    def __init__(self, device, ns, nt, src_group, trg_group, exclude_same_group, n_groups):
        if exclude_same_group is None:
            exclude_same_group = src_group is not None and trg_group is not None
        self.tensors = []
        if not exclude_same_group:
            self.ex = None
            return
        if src_group is None or trg_group is None:
            raise ValueError("exclude_same_group needs src_group and trg_group")
        sg = _vec1(src_group, ns, "src_group", device, torch.int32)
        tg = _vec1(trg_group, nt, "trg_group", device, torch.int32)
        if n_groups is None:   # one synchronisation: the largest id
            n_groups = 1 + int(max(int(sg.max()) if ns else -1, int(tg.max()) if nt else -1, 0))
        self.tensors = [sg, tg]
        self.ex = C.Exclusion(C.EXCL_SAME_GROUP, _ptr(sg).value, _ptr(tg).value, None, int(n_groups), 0.0)

    def ref(self):
        return ctypes.byref(self.ex) if self.ex is not None else None


def _fmm_common(plan, device, ns, nt, depth, rule):
    size = ctypes.c_size_t()
    C.check(C.lib().stokes_fmm_workspace_size(context(device), plan.handle, ns, nt, int(depth), rule.ref(),
                                              ctypes.byref(size)))
    return torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=device), int(size.value)


def fmm_sl(plan, src, f, w, trg, centre, half_width, depth, mu=1.0, out=None, accumulate=False, precision="fp64",
           src_group=None, trg_group=None, exclude_same_group=None, n_groups=None):
    """Single-layer sum by the FMM; see stokes_fmm_sl_eval.  precision "mixed"
    runs the near-field pairs in float32.  With src_group and trg_group the
    same-group rule applies (ids in [0, n_groups); n_groups defaults to the
    largest id + 1, which costs one synchronisation)."""
    device = src.device
    _vec3(src, "src", device); _vec3(f, "f", device); _vec3(trg, "trg", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    out = _out(out, nt, device, accumulate)
    rule = _FmmRule(device, ns, nt, src_group, trg_group, exclude_same_group, n_groups)
    ws, size = _fmm_common(plan, device, ns, nt, depth, rule)
    c = (ctypes.c_double * 3)(*[float(v) for v in centre])
    opts = C.Opts(_fmm_precision(precision), int(bool(accumulate)))
    C.check(C.lib().stokes_fmm_sl_eval(context(device), plan.handle, ns, _ptr(src), _ptr(f), _ptr(w), nt, _ptr(trg),
                                       float(mu), c, float(half_width), int(depth), rule.ref(), ctypes.byref(opts),
                                       _ptr(out), _ptr(ws), size, _stream(device)))
    return out


def fmm_dl(plan, src, phi, w, nrm, trg, centre, half_width, depth, out=None, accumulate=False, precision="fp64",
           src_group=None, trg_group=None, exclude_same_group=None, n_groups=None):
    """Double-layer sum by the FMM; see stokes_fmm_dl_eval.  precision "mixed"
    runs the near-field pairs in float32; the pair rule as in fmm_sl."""
    device = src.device
    _vec3(src, "src", device); _vec3(phi, "phi", device); _vec3(nrm, "nrm", device); _vec3(trg, "trg", device)
    ns, nt = src.shape[1], trg.shape[1]
    _vec1(w, ns, "w", device)
    out = _out(out, nt, device, accumulate)
    rule = _FmmRule(device, ns, nt, src_group, trg_group, exclude_same_group, n_groups)
    ws, size = _fmm_common(plan, device, ns, nt, depth, rule)
    c = (ctypes.c_double * 3)(*[float(v) for v in centre])
    opts = C.Opts(_fmm_precision(precision), int(bool(accumulate)))
    C.check(C.lib().stokes_fmm_dl_eval(context(device), plan.handle, ns, _ptr(src), _ptr(phi), _ptr(w), _ptr(nrm), nt,
                                       _ptr(trg), c, float(half_width), int(depth), rule.ref(), ctypes.byref(opts),
                                       _ptr(out), _ptr(ws), size, _stream(device)))
    return out

