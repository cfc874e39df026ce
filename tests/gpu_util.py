"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np
import torch

FP64_TOL = 1e-12      # relative L2 bound for the float64 path
MIXED_TOL = 1e-6      # relative L2 bound for the mixed float32/float64 path


def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda", 0)


def dev(a, d=None, dtype=None):
    d = d or device()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(d)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_close(got, ref, tol, what=""):
    """Relative L2 within tol, and every element within 10 tol of the largest
    reference magnitude (no single element may hide behind the average)."""
    assert got.shape == ref.shape, (got.shape, ref.shape)
    r = rel_l2(got, ref)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    assert r <= tol, f"{what}: rel-L2 {r:.3e} > {tol:.1e}"
    emax = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
    assert emax <= 10 * tol, f"{what}: max elementwise error {emax:.3e} > {10 * tol:.1e}"
    return r
