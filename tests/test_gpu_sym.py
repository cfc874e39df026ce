"""GPU parity of the each-pair-once single-layer sum over shared point sets
(the Stokeslet's symmetry, eq. sl_stokes) against the FP64 oracle: ragged
sizes around the 64-point tiles and 1024-point row blocks, cell-ordered and
shuffled groups, coincident points within and across tiles, the rule on and
off, accumulation, stream-K cuts at every unit boundary, the fallback to
one-sided evaluation with a smaller workspace, and run-to-run identity."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1909_11085_amd as S
from oracle import oracle as O
from paper_1909_11085_amd import _capi as C
from paper_1909_11085_amd import workloads as W
from tests.gpu_util import FP64_TOL, MIXED_TOL, assert_close, dev, device, host

TOL = {"fp64": FP64_TOL, "mixed": MIXED_TOL}

pytestmark = pytest.mark.gpu


def _shared(seed, n, layout="cells", dup=6):
    """n points in clusters of 544 (cell order), or shuffled, with groups."""
    rng = np.random.default_rng(seed)
    n_cells = max(1, (n + 543) // 544)
    centres = rng.uniform(-12.0, 12.0, (n_cells, 3))
    g = np.minimum(np.arange(n) // 544, n_cells - 1).astype(np.int32)
    pos = (centres[g] + 2.0 * rng.standard_normal((n, 3))).T.copy()
    if layout == "shuffled":
        perm = rng.permutation(n)
        pos, g = pos[:, perm].copy(), g[perm].copy()
    if dup and n > 2 * dup:
        src = rng.choice(n, dup, replace=False)
        dst = rng.choice(np.setdiff1d(np.arange(n), src), dup, replace=False)
        pos[:, dst] = pos[:, src]                          # coincident points, any groups
    return pos, rng.standard_normal((3, n)), rng.uniform(0.1, 1.0, n), g


def _run(pos, f, w, g, excl, precision="fp64", **kw):
    P, G = dev(pos), dev(g)
    if precision == "mixed":
        kw.setdefault("group_h", dev(np.full(int(g.max()) + 1, 0.45)))
    return S.sl(P, dev(f), dev(w), P, src_group=G, trg_group=G, exclude_same_group=excl, precision=precision,
                **kw)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 1023, 1024, 1025, 2049, 5000, 17_000])
@pytest.mark.parametrize("excl", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ragged_sizes(n, excl, precision):
    print(f"case sym n={n} excl={excl} {precision}", flush=True)
    pos, f, w, g = _shared(100 + n, n)
    got = host(_run(pos, f, w, g, excl, precision, mu=0.9))
    ref = O.sl(pos, f, w, pos, mu=0.9, src_group=g, trg_group=g, exclude_same_group=excl)
    assert_close(got, ref, TOL[precision], f"sym n={n} {precision}")


@pytest.mark.parametrize("layout", ["cells", "shuffled"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_layouts_and_one_sided_agree(layout, precision):
    """Shuffled groups defeat every group-range test (most units take the
    masked loop); the one-sided path (pair symmetry off) agrees."""
    pos, f, w, g = _shared(7, 9_000, layout)
    ref = O.sl(pos, f, w, pos, src_group=g, trg_group=g, exclude_same_group=True)
    got = host(_run(pos, f, w, g, True, precision))
    assert_close(got, ref, TOL[precision], layout)
    S.set_pair_symmetry(False)
    try:
        one = host(_run(pos, f, w, g, True, precision))
    finally:
        S.set_pair_symmetry(True)
    assert_close(one, ref, TOL[precision], layout + " one-sided")


@pytest.mark.parametrize("grid", [1, 3, 7, 64, 1000])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stream_k_cuts(grid, precision):
    """Forced workgroup counts cut the unit triangle at other places (ranges
    inside one row block, ranges spanning many)."""
    pos, f, w, g = _shared(8, 6_000)
    ref = O.sl(pos, f, w, pos, src_group=g, trg_group=g, exclude_same_group=True)
    S.set_grid_override(grid)
    try:
        got = host(_run(pos, f, w, g, True, precision))
    finally:
        S.set_grid_override(0)
    assert_close(got, ref, TOL[precision], f"grid={grid}")


def test_accumulate_and_identity():
    pos, f, w, g = _shared(9, 4_100)
    base = np.random.default_rng(10).standard_normal((3, 4_100))
    out = dev(base.copy())
    _run(pos, f, w, g, True, out=out, accumulate=True)
    ref = O.sl(pos, f, w, pos, src_group=g, trg_group=g, exclude_same_group=True)
    assert_close(host(out) - base, ref, FP64_TOL, "accumulate")
    a, b = host(_run(pos, f, w, g, True)), host(_run(pos, f, w, g, True))
    assert np.array_equal(a, b)                           # no atomics: bitwise the same


def test_small_workspace_takes_the_one_sided_path():
    """Through the C ABI: a workspace of the one-sided size (smaller than the
    shared-set size that stokes_workspace_size reports) still gives the sum."""
    n = 3_000
    pos, f, w, g = _shared(11, n)
    P, F, Wt, G = dev(pos), dev(f), dev(w), dev(g)
    L, ctx = C.lib(), S.context()
    op, size_sh = C.Opts(C.FP64, 0), ctypes.c_size_t()
    assert L.stokes_workspace_size(ctx, C.OP_SL, n, n, 0, 0, ctypes.byref(op), ctypes.byref(size_sh)) == C.OK
    size_1 = ctypes.c_size_t()
    assert L.stokes_workspace_size(ctx, C.OP_SL, n, n + 1, 0, 0, ctypes.byref(op), ctypes.byref(size_1)) == C.OK
    assert size_sh.value > size_1.value
    ws = torch.empty(size_1.value, dtype=torch.uint8, device=device())
    out = torch.empty((3, n), dtype=torch.float64, device=device())
    ex = C.Exclusion(C.EXCL_SAME_GROUP, G.data_ptr(), G.data_ptr(), 0, 0, 0.5)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = L.stokes_sl_eval(ctx, n, vp(P), vp(F), vp(Wt), n, vp(P), 1.0, ctypes.byref(ex), ctypes.byref(op),
                          vp(out), vp(ws), size_1.value, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == C.OK, L.stokes_last_error()
    ref = O.sl(pos, f, w, pos, src_group=g, trg_group=g, exclude_same_group=True)
    assert_close(host(out), ref, FP64_TOL, "one-sided fallback")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cells_workload_sampled(precision):
    """512 cells (278,528 points), the benchmark's launch: 512 seeded points
    against the oracle."""
    cfg = W.make_config(2)
    c, f = cfg["cells"], cfg["f"]
    got = host(_run(c.pos, f, c.weight, c.group, True, precision, group_h=dev(c.group_h)))
    idx = W.subset(np.random.default_rng(222), c.n, 512)
    ref = O.sl(c.pos, f, c.weight, c.pos[:, idx], src_group=c.group, trg_group=c.group[idx],
               exclude_same_group=True)
    r = assert_close(got[:, idx], ref, TOL[precision], f"cfg2 sym {precision}")
    print(f"cfg2 each-pair-once {precision} rel-L2 {r:.3e}")


# ---------------------------------------------------------------- adjoint
def _vjp(pos, f, w, g, gu, excl, grad_f=True, grad_x=True, accumulate=False, base=None):
    P, G, n = dev(pos), dev(g), pos.shape[1]
    gf = dev(base[0].copy()) if base is not None else (dev(np.zeros((3, n))) if grad_f else None)
    gx = dev(base[1].copy()) if base is not None else (dev(np.zeros((3, n))) if grad_x else None)
    S.sl_vjp(P, dev(f), dev(w), P, dev(gu), mu=1.1, src_group=G, trg_group=G, exclude_same_group=excl,
             grad_f=gf if grad_f else None, grad_src=gx if grad_x else None, grad_trg=gx if grad_x else None,
             accumulate=accumulate)
    return (host(gf) if grad_f else None), (host(gx) if grad_x else None)


def _vjp_ref(pos, f, w, g, gu, excl):
    rf, rs, rt = O.sl_vjp(pos, f, w, pos, gu, mu=1.1, src_group=g, trg_group=g, exclude_same_group=excl)
    return rf, rs + rt


@pytest.mark.parametrize("n", [1, 63, 65, 1023, 1025, 3000, 9000])
@pytest.mark.parametrize("excl", [True, False])
def test_adjoint_ragged_sizes(n, excl):
    """dL/df and the total dL/dx on a shared point set (one combined position
    gradient): the each-pair-once adjoint against the oracle."""
    print(f"case sym adjoint n={n} excl={excl}", flush=True)
    pos, f, w, g = _shared(300 + n, n)
    gu = np.random.default_rng(301 + n).standard_normal((3, n))
    gf, gx = _vjp(pos, f, w, g, gu, excl)
    rf, rx = _vjp_ref(pos, f, w, g, gu, excl)
    assert_close(gf, rf, FP64_TOL, f"adjoint dL/df n={n}")
    assert_close(gx, rx, FP64_TOL, f"adjoint dL/dx n={n}")


@pytest.mark.parametrize("layout", ["cells", "shuffled"])
def test_adjoint_layouts_one_sided_and_outputs(layout):
    """Shuffled groups (most units masked); the one-sided fused pass agrees;
    either output alone; accumulation."""
    n = 5000
    pos, f, w, g = _shared(17, n, layout)
    gu = np.random.default_rng(18).standard_normal((3, n))
    rf, rx = _vjp_ref(pos, f, w, g, gu, True)
    gf, gx = _vjp(pos, f, w, g, gu, True)
    assert_close(gf, rf, FP64_TOL, layout + " dL/df")
    assert_close(gx, rx, FP64_TOL, layout + " dL/dx")
    assert_close(_vjp(pos, f, w, g, gu, True, grad_f=False)[1], rx, FP64_TOL, "dL/dx alone")
    base = np.random.default_rng(19).standard_normal((2, 3, n))
    af, ax = _vjp(pos, f, w, g, gu, True, accumulate=True, base=base)
    assert_close(af - base[0], rf, FP64_TOL, "accumulated dL/df")
    assert_close(ax - base[1], rx, FP64_TOL, "accumulated dL/dx")
    S.set_pair_symmetry(False)
    try:
        of, ox = _vjp(pos, f, w, g, gu, True)
    finally:
        S.set_pair_symmetry(True)
    assert_close(of, rf, FP64_TOL, "one-sided dL/df")
    assert_close(ox, rx, FP64_TOL, "one-sided dL/dx")


@pytest.mark.parametrize("grid", [1, 5, 333])
def test_adjoint_stream_k_cuts(grid):
    n = 4500
    pos, f, w, g = _shared(21, n)
    gu = np.random.default_rng(22).standard_normal((3, n))
    rf, rx = _vjp_ref(pos, f, w, g, gu, True)
    S.set_grid_override(grid)
    try:
        gf, gx = _vjp(pos, f, w, g, gu, True)
    finally:
        S.set_grid_override(0)
    assert_close(gf, rf, FP64_TOL, f"grid={grid} dL/df")
    assert_close(gx, rx, FP64_TOL, f"grid={grid} dL/dx")
    a, b = _vjp(pos, f, w, g, gu, True), _vjp(pos, f, w, g, gu, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])     # no atomics
