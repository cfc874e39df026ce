"""GPU parity of the direct single- and double-layer sums against the FP64 oracle.

Every case calls the HIP library through the C ABI (via the thin binding) and
compares it with the oracle on the same seeded inputs: in full where the oracle
finishes in seconds, and on seeded target samples (same launch as the
benchmark: all targets computed, a subset checked) at the full workload sizes.
"""
import math

import numpy as np
import pytest
import torch

import paper_1909_11085_amd as S
from oracle import oracle as O
from paper_1909_11085_amd import workloads as W
from tests.gpu_util import FP64_TOL, MIXED_TOL, assert_close, dev, device, host, rel_l2

pytestmark = pytest.mark.gpu

PREC_TOL = {"fp64": FP64_TOL, "mixed": MIXED_TOL}


def _cloud(seed, ns, nt, n_groups=5, dup=8, spread=6.0):
    """Clustered random points with groups; `dup` targets coincide with sources."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-spread, spread, (n_groups, 3))
    gs = rng.integers(0, n_groups, ns).astype(np.int32)
    y = (centres[gs] + rng.standard_normal((ns, 3))).T.copy()
    gt = rng.integers(0, n_groups, nt).astype(np.int32)
    x = (centres[gt] + rng.standard_normal((nt, 3))).T.copy()
    if dup and nt >= dup and ns >= dup:
        x[:, :dup] = y[:, :dup]
        gt[:dup] = gs[:dup]
    f = rng.standard_normal((3, ns))
    w = rng.uniform(0.1, 1.0, ns)
    nv = rng.standard_normal((3, ns))
    nv /= np.linalg.norm(nv, axis=0)
    h = rng.uniform(0.2, 0.6, n_groups)
    return dict(y=y, x=x, f=f, w=w, n=nv, gs=gs, gt=gt, h=h)


def _run(kernel, c, precision, excl, mu=1.0, near_frac=0.5, out=None, accumulate=False):
    d = device()
    kw = dict(src_group=dev(c["gs"]), trg_group=dev(c["gt"]), exclude_same_group=excl,
              precision=precision, group_h=dev(c["h"]), near_frac=near_frac, out=out,
              accumulate=accumulate)
    if kernel == "sl":
        return S.sl(dev(c["y"]), dev(c["f"]), dev(c["w"]), dev(c["x"]), mu=mu, **kw)
    return S.dl(dev(c["y"]), dev(c["f"]), dev(c["w"]), dev(c["n"]), dev(c["x"]), **kw)


def _oracle(kernel, c, excl, mu=1.0):
    kw = dict(src_group=c["gs"], trg_group=c["gt"], exclude_same_group=excl)
    if kernel == "sl":
        return O.sl(c["y"], c["f"], c["w"], c["x"], mu=mu, **kw)
    return O.dl(c["y"], c["f"], c["w"], c["n"], c["x"], **kw)


@pytest.mark.parametrize("kernel", ["sl", "dl"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("excl", [True, False])
@pytest.mark.parametrize("sizes", [(1000, 777), (257, 1), (1, 300), (3001, 2049)])
def test_ragged_clouds(kernel, precision, excl, sizes):
    print(f"case kernel={kernel} precision={precision} excl={excl} sizes={sizes}", flush=True)
    c = _cloud(7 + sizes[0], *sizes)
    got = host(_run(kernel, c, precision, excl, mu=1.7))
    ref = _oracle(kernel, c, excl, mu=1.7)
    assert_close(got, ref, PREC_TOL[precision], f"{kernel}/{precision}/{excl}/{sizes}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg1_full(precision):
    """8 Evans-Fung cells, 4,352 points, all points are targets, same-cell rule."""
    print(f"case cfg1 precision={precision}", flush=True)
    cfg = W.make_config(1)
    cells, f = cfg["cells"], cfg["f"]
    d = device()
    u = S.sl(dev(cells.pos), dev(f), dev(cells.weight), dev(cells.pos), mu=1.0,
             src_group=dev(cells.group), trg_group=dev(cells.group), precision=precision,
             group_h=dev(cells.group_h), near_frac=0.5)
    ref = O.sl(cells.pos, f, cells.weight, cells.pos, src_group=cells.group,
               trg_group=cells.group, exclude_same_group=True)
    r = assert_close(host(u), ref, PREC_TOL[precision], f"cfg1/{precision}")
    print(f"cfg1 {precision} rel-L2 {r:.3e}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("grid", [1, 2, 3, 7, 64, 1000])
def test_work_partition_agrees(grid, precision):
    """Any workgroup count (stream-K ranges cutting target blocks anywhere)
    gives the same sums within the bound."""
    c = _cloud(99, 5000, 2600)
    ref = _oracle("sl", c, True)
    try:
        S.set_grid_override(grid)
        got = host(_run("sl", c, precision, True))
    finally:
        S.set_grid_override(0)
    assert_close(got, ref, PREC_TOL[precision], f"grid={grid}/{precision}")


def test_fp64_is_deterministic():
    c = _cloud(5, 20000, 9000)
    a = host(_run("sl", c, "fp64", True))
    b = host(_run("sl", c, "fp64", True))
    assert np.array_equal(a, b)


def test_accumulate_superposes():
    """u = D[phi] + S[f] at the same targets through the accumulate flag."""
    c = _cloud(17, 2000, 1500)
    u = _run("dl", c, "fp64", False)
    _run("sl", c, "fp64", True, mu=0.6, out=u, accumulate=True)
    ref = _oracle("dl", c, False) + _oracle("sl", c, True, mu=0.6)
    assert_close(host(u), ref, FP64_TOL, "accumulate")


@pytest.mark.parametrize("kernel", ["sl", "dl"])
def test_empty_sources_and_targets(kernel):
    d = device()
    c = _cloud(3, 10, 10)
    z3 = torch.zeros((3, 0), dtype=torch.float64, device=d)
    z1 = torch.zeros(0, dtype=torch.float64, device=d)
    x = dev(c["x"])
    if kernel == "sl":
        u = S.sl(z3, z3, z1, x)
    else:
        u = S.dl(z3, z3, z1, z3, x)
    assert host(u).shape == (3, 10) and np.all(host(u) == 0.0)
    prev = torch.full((3, 10), 2.5, dtype=torch.float64, device=d)
    if kernel == "sl":
        S.sl(z3, z3, z1, x, out=prev, accumulate=True)
    else:
        S.dl(z3, z3, z1, z3, x, out=prev, accumulate=True)
    assert np.all(host(prev) == 2.5)
    if kernel == "sl":
        u0 = S.sl(dev(c["y"]), dev(c["f"]), dev(c["w"]), z3)
    else:
        u0 = S.dl(dev(c["y"]), dev(c["f"]), dev(c["w"]), dev(c["n"]), z3)
    assert u0.shape == (3, 0)


def test_sphere_closed_form_on_gpu():
    """Uniform traction on a sphere gives the rigid velocity 2 a f/(3 mu) inside."""
    a, mu = 1.7, 0.8
    p, w, n = W.sphere_surface(a, order=32)
    fvec = np.array([0.3, -1.1, 0.6])
    f = np.repeat(fvec[:, None], p.shape[1], axis=1)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, 100))
    x = v / np.linalg.norm(v, axis=0) * rng.uniform(0, 0.5 * a, 100)
    u = host(S.sl(dev(p), dev(f), dev(w), dev(x), mu=mu))
    expect = np.repeat((2 * a * fvec / (3 * mu))[:, None], 100, axis=1)
    assert rel_l2(u, expect) < 1e-13
    # double-layer Gauss identity: the constant density f gives -f inside
    ud = host(S.dl(dev(p), dev(f), dev(w), dev(n), dev(x)))
    assert rel_l2(ud, -np.repeat(fvec[:, None], 100, axis=1)) < 1e-12


def test_mixed_translation_invariance():
    """Shifting all points by (1e3, -2e3, 5e2): the mixed path stays within its
    tolerance of the unshifted FP64 oracle (tile-centred float32 offsets)."""
    cfg = W.make_config(1)
    cells, f = cfg["cells"], cfg["f"]
    shift = np.array([1e3, -2e3, 5e2])[:, None]
    ref = O.sl(cells.pos, f, cells.weight, cells.pos, src_group=cells.group,
               trg_group=cells.group, exclude_same_group=True)
    pos = cells.pos + shift
    u = S.sl(dev(pos), dev(f), dev(cells.weight), dev(pos), src_group=dev(cells.group),
             trg_group=dev(cells.group), precision="mixed", group_h=dev(cells.group_h))
    assert_close(host(u), ref, MIXED_TOL, "mixed shifted")


# ---------------------------------------------------------------- full-size workloads
@pytest.fixture(scope="module")
def cfg2():
    return W.make_config(2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg2_sampled(cfg2, precision):
    """512 cells, 278,528 points: the benchmark's launch, 512 seeded targets checked."""
    print(f"case cfg2 precision={precision}", flush=True)
    cells, f = cfg2["cells"], cfg2["f"]
    u = S.sl(dev(cells.pos), dev(f), dev(cells.weight), dev(cells.pos), src_group=dev(cells.group),
             trg_group=dev(cells.group), precision=precision, group_h=dev(cells.group_h),
             near_frac=0.5)
    idx = W.subset(np.random.default_rng(2002), cells.n, 512)
    ref = O.sl(cells.pos, f, cells.weight, cells.pos[:, idx], src_group=cells.group,
               trg_group=cells.group[idx], exclude_same_group=True)
    r = assert_close(host(u)[:, idx], ref, PREC_TOL[precision], f"cfg2/{precision}")
    print(f"cfg2 {precision} rel-L2 on 512 targets {r:.3e}")


@pytest.fixture(scope="module")
def cfg5():
    return W.make_config(5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg5_wall_double_layer_sampled(cfg5, precision):
    """1,048,576 wall points -> 522,240 cell points, 256 seeded targets checked."""
    print(f"case cfg5 DL precision={precision}", flush=True)
    wall, cells, phi = cfg5["wall"], cfg5["cells"], cfg5["phi"]
    u = S.dl(dev(wall.pos), dev(phi), dev(wall.weight), dev(wall.normal), dev(cells.pos),
             src_group=dev(wall.group), precision=precision, group_h=dev(wall.group_h),
             near_frac=0.5, exclude_same_group=False)
    idx = W.subset(np.random.default_rng(5005), cells.n, 256)
    ref = O.dl(wall.pos, phi, wall.weight, wall.normal, cells.pos[:, idx])
    r = assert_close(host(u)[:, idx], ref, PREC_TOL[precision], f"cfg5-DL/{precision}")
    print(f"cfg5 DL {precision} rel-L2 on 256 targets {r:.3e}")


def _rotation(seed):
    q = np.random.default_rng(seed).standard_normal(4)
    a, b, c, d = q / np.linalg.norm(q)
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


@pytest.mark.parametrize("kernel", ["sl", "dl"])
def test_rotation_equivariance_on_gpu(kernel):
    """u(Qx; Qy, Q f, Q n) = Q u(x; y, f, n): both sums are built from r, r.q,
    r.n and rho only, so rotating every vector rotates the result."""
    c = _cloud(31, 900, 700, dup=0)
    Q = _rotation(5)
    cr = dict(c, y=Q @ c["y"], x=Q @ c["x"], f=Q @ c["f"], n=Q @ c["n"])
    u = host(_run(kernel, c, "fp64", True))
    ur = host(_run(kernel, cr, "fp64", True))
    assert rel_l2(ur, Q @ u) < 1e-13


def test_symmetry_of_weighted_single_layer_on_gpu():
    """The Stokeslet is symmetric, S(x, y) = S(y, x) = S^T, so on a shared point
    set with the same-group rule <w g, A f> = <w f, A g> with (A f)_n = sum_m S w_m f_m."""
    cfg = W.make_config(1)
    cells = cfg["cells"]
    rng = np.random.default_rng(17)
    f, g = rng.standard_normal((2, 3, cells.n))
    p, w, gr = dev(cells.pos), dev(cells.weight), dev(cells.group)
    af = host(S.sl(p, dev(f), w, p, src_group=gr, trg_group=gr))
    ag = host(S.sl(p, dev(g), w, p, src_group=gr, trg_group=gr))
    lhs = float(np.sum(cells.weight * g * af))
    rhs = float(np.sum(cells.weight * f * ag))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_linearity_and_viscosity_on_gpu(precision):
    """u(alpha f) = alpha u(f); the single layer scales as 1/mu and the double
    layer does not depend on mu (it takes none)."""
    c = _cloud(41, 1200, 800, dup=0)
    u1 = host(_run("sl", c, precision, True, mu=1.0))
    u2 = host(_run("sl", dict(c, f=-2.5 * c["f"]), precision, True, mu=4.0))
    assert rel_l2(u2, -2.5 / 4.0 * u1) < PREC_TOL[precision]
    d1 = host(_run("dl", c, precision, True))
    d2 = host(_run("dl", dict(c, f=3.0 * c["f"]), precision, True))
    assert rel_l2(d2, 3.0 * d1) < PREC_TOL[precision]
