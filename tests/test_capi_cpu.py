"""C-ABI contract checks that run without a GPU: the library loads, exports
every function the header declares, and rejects bad arguments before any
device work (no compute calls are made here)."""
import ctypes

import pytest

from paper_1909_11085_amd import _capi as C


def test_exports_every_declared_function():
    lib = C.lib()
    names = C.header_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(C._SIGNATURES), set(names) ^ set(C._SIGNATURES)


def test_version():
    assert C.lib().stokes_version() == 10000


def test_create_reports_device_status():
    h = ctypes.c_void_p()
    rc = C.lib().stokes_create(ctypes.byref(h), 0)
    if rc == C.OK:           # a GPU is present: release it
        C.lib().stokes_destroy(h)
        pytest.skip("a device is present; the no-device path is not reachable here")
    assert rc in (C.EDEVICE, C.EUNSUPPORTED)
    assert h.value is None
    assert C.lib().stokes_last_error()


def test_null_context_is_rejected():
    L = C.lib()
    ex, op = C.Exclusion(), C.Opts()
    rc = L.stokes_sl_eval(None, 0, None, None, None, 0, None, 1.0, ctypes.byref(ex),
                          ctypes.byref(op), None, None, 0, None)
    assert rc == C.EINVAL
    assert b"ctx" in L.stokes_last_error()
    size = ctypes.c_size_t()
    assert L.stokes_workspace_size(None, C.OP_SL, 10, 10, 0, 0, None, ctypes.byref(size)) == C.EINVAL
    assert L.stokes_set_grid_override(None, 2) == C.EINVAL
    assert L.stokes_create(None, 0) == C.EINVAL
    L.stokes_destroy(None)          # no-op
    L.stokes_p2p_plan_destroy(None)  # no-op


def test_bad_mu_is_rejected_before_anything_else():
    L = C.lib()
    for mu in (0.0, -1.0, float("nan"), float("inf")):
        rc = L.stokes_sl_eval(None, 0, None, None, None, 0, None, mu, None, None, None, None, 0, None)
        assert rc == C.EINVAL
        assert b"mu" in L.stokes_last_error()
