"""ctypes binding of the C ABI in ``include/stokes_mi355x.h``.

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly when ``libstokes_mi355x.so`` has not been built; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstokes_mi355x.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "stokes_mi355x.h")

OK, EINVAL, EDEVICE, ELAUNCH, EWORKSPACE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
EXCL_NONE, EXCL_SAME_GROUP = 0, 1
KERNEL_SL, KERNEL_DL = 0, 1
OP_SL, OP_DL, OP_P2P_SL, OP_P2P_DL, OP_SL_VJP, OP_DL_VJP, OP_P2P_SL_VJP, OP_P2P_DL_VJP = range(8)
NOALLOC_SCRATCH_BYTES = 64 << 20
PAIR_F32, PAIR_F64, PAIR_SKIP = 1, 1 << 8, 1 << 16
STATUS_NAMES = {OK: "STOKES_OK", EINVAL: "STOKES_EINVAL", EDEVICE: "STOKES_EDEVICE",
                ELAUNCH: "STOKES_ELAUNCH", EWORKSPACE: "STOKES_EWORKSPACE",
                EUNSUPPORTED: "STOKES_EUNSUPPORTED"}


class StokesError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Exclusion(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("src_group", ctypes.c_void_p),
                ("trg_group", ctypes.c_void_p), ("group_h", ctypes.c_void_p),
                ("n_groups", ctypes.c_int32), ("near_frac", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("accumulate", ctypes.c_int32)]


class PatchRule(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("eta", ctypes.c_int32), ("p", ctypes.c_int32),
                ("R_frac", ctypes.c_double), ("r_frac", ctypes.c_double),
                ("nodes_1d", ctypes.POINTER(ctypes.c_double)),
                ("weights_1d", ctypes.POINTER(ctypes.c_double))]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_EX = ctypes.POINTER(Exclusion)
_OP = ctypes.POINTER(Opts)
_PR = ctypes.POINTER(PatchRule)

_SIGNATURES = {
    "stokes_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "stokes_destroy": (None, [_vp]),
    "stokes_last_error": (ctypes.c_char_p, []),
    "stokes_version": (ctypes.c_int, []),
    "stokes_set_grid_override": (ctypes.c_int, [_vp, _i32]),
    "stokes_set_pair_symmetry": (ctypes.c_int, [_vp, _i32]),
    "stokes_debug_pair_classes": (ctypes.c_int, [_vp, _vp, _i64, _i64]),
    "stokes_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "stokes_timing_read": (ctypes.c_int, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
    "stokes_workspace_size": (ctypes.c_int, [_vp, _i32, _i64, _i64, _i32, _i64, _OP, ctypes.POINTER(_sz)]),
    "stokes_sl_eval": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _i64, _vp, _dbl, _EX, _OP, _vp,
                                      _vp, _sz, _vp]),
    "stokes_sl_eval_noalloc": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _i64, _vp, _dbl, _EX, _OP,
                                              _vp, _vp]),
    "stokes_dl_eval": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _EX, _OP, _vp,
                                      _vp, _sz, _vp]),
    "stokes_p2p_plan_create": (ctypes.c_int, [_vp, _i32, _i64, _i64, _vp, _vp, _vp, _vp, _i64,
                                              ctypes.POINTER(_vp)]),
    "stokes_p2p_plan_destroy": (None, [_vp]),
    "stokes_p2p_plan_pairs": (ctypes.c_int, [_vp, ctypes.POINTER(_i64)]),
    "stokes_p2p_plan_eval": (ctypes.c_int, [_vp, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _i64, _vp,
                                            _dbl, _EX, _OP, _vp, _vp, _sz, _vp]),
    "stokes_p2p_leaf_eval": (ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp,
                                            _vp, _vp, _i64, _dbl, _EX, _OP, _vp, _vp, _sz, _vp]),
    "stokes_sl_vjp": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _i64, _vp, _dbl, _EX, _OP, _vp,
                                     _vp, _vp, _vp, _vp, _sz, _vp]),
    "stokes_dl_vjp": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _EX, _OP, _vp,
                                     _vp, _vp, _vp, _vp, _sz, _vp]),
    "stokes_p2p_sl_vjp": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp, _i64,
                                         _dbl, _EX, _OP, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "stokes_p2p_dl_vjp": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp, _vp, _i64,
                                         _EX, _OP, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "stokes_patch_upsample": (ctypes.c_int, [_vp, _i64, _PR, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "stokes_checkpoint_workspace_size": (ctypes.c_int, [_vp, _i64, _PR, _i64, _OP, ctypes.POINTER(_sz)]),
    "stokes_dl_checkpoint_eval": (ctypes.c_int, [_vp, _i64, _PR, _vp, _vp, _i64, _vp, _vp, _OP, _vp, _vp,
                                                 _vp, _vp, _sz, _vp]),
    "stokes_bie_workspace_size": (ctypes.c_int, [_vp, _i64, _PR, _i32, _OP, ctypes.POINTER(_sz)]),
    "stokes_bie_apply": (ctypes.c_int, [_vp, _i64, _PR, _vp, _vp, _OP, _vp, _vp, _sz, _vp]),
    "stokes_bie_solve": (ctypes.c_int, [_vp, _i64, _PR, _vp, _vp, _i32, _dbl, _OP, _vp,
                                        ctypes.POINTER(_i32), ctypes.POINTER(_dbl), _vp, _sz, _vp]),
    "stokes_space_time_boxes": (ctypes.c_int, [_vp, _i32, _vp, _i64, _vp, _vp, _dbl, _vp, _vp, _vp]),
    "stokes_collision_workspace_size": (ctypes.c_int, [_vp, _i32, _i64, ctypes.POINTER(_sz)]),
    "stokes_collision_candidates": (ctypes.c_int, [_vp, _i32, _vp, _vp, _dbl, _i64, _vp, _i64,
                                                   ctypes.POINTER(_i64), ctypes.POINTER(_i64), _vp, _sz, _vp]),
    "stokes_fmm_plan_create": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_vp)]),
    "stokes_fmm_plan_destroy": (None, [_vp]),
    "stokes_fmm_workspace_size": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i32, _EX, ctypes.POINTER(_sz)]),
    "stokes_fmm_sl_eval": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _dbl, _vp, _dbl, _i32, _EX,
                                          _OP, _vp, _vp, _sz, _vp]),
    "stokes_fmm_dl_eval": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _dbl, _i32, _EX,
                                          _OP, _vp, _vp, _sz, _vp]),
}

_lib = None


def header_functions():
    """Names of the functions that the public header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stokes_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status):
    if status != OK:
        msg = lib().stokes_last_error()
        raise StokesError(status, msg.decode() if msg else "")
    return status
