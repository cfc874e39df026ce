"""GPU parity of the spatial-hash collision-candidate search (Sec. 4, steps a-c
of Sec. 3.3) against the CPU oracle.  Boxes are min / max of the inputs and the
cells floor((x - origin) / H) in float64 on both sides, so boxes and pairs
must agree exactly (bit for bit, and pair for pair in the documented order)."""
import ctypes
import math

import numpy as np
import pytest
import torch

import paper_1909_11085_amd as S
from oracle import spatial as SP
from paper_1909_11085_amd import _capi as C
from paper_1909_11085_amd import workloads as W
from tests.gpu_util import dev, device, host

pytestmark = pytest.mark.gpu


def _expected_order(pairs, lo, hi, H):
    """Oracle pairs in the library's order: Morton key of the pair's lowest
    shared cell, then i, then j."""
    clo, _ = SP.cell_ranges(lo, hi, H)
    keys = [SP.morton3(*np.maximum(clo[:, i], clo[:, j])) for i, j in pairs]
    order = sorted(range(len(pairs)), key=lambda k: (keys[k], pairs[k][0], pairs[k][1]))
    return np.asarray(pairs, dtype=np.int64).reshape(-1, 2)[order]


def _check(lo, hi, H, **kw):
    got = host(S.collision_candidates(dev(lo), dev(hi), H, **kw)).T.astype(np.int64)
    ref = SP.collision_candidates(lo, hi, H)
    assert np.array_equal(got, _expected_order(ref, lo, hi, H)), (len(got), len(ref))
    return got


def test_space_time_boxes_match_oracle():
    cfg = W.make_config(1)
    cells = cfg["cells"]
    rng = np.random.default_rng(61)
    x1 = W.cells_after_step(rng, cells)
    ofs = W.group_offsets(cells.group)
    ofs = np.concatenate([ofs[:3], ofs[2:3], ofs[3:]])          # an empty mesh as mesh 2
    for x1_ in (x1, None):
        for inflate in (0.0, 0.37):
            lo, hi = S.space_time_boxes(dev(ofs), dev(cells.pos), None if x1_ is None else dev(x1_), inflate)
            rlo, rhi = SP.space_time_boxes(cells.pos, x1_, ofs, inflate)
            assert np.array_equal(host(lo), rlo) and np.array_equal(host(hi), rhi)


def test_golden_boxes():
    lo = np.array([[0.0, 0.6, 1.5, 0.2, 0.0, 0.25, 0.5], [0.0, 0.2, 0.1, 1.5, 0.0, 0.25, 0.6],
                   [0.0, 0.2, 0.1, 0.2, 3.0, 0.25, 0.0]])
    hi = np.array([[0.5, 1.2, 2.5, 0.3, 2.9, 0.26, 1.0], [0.5, 0.4, 0.3, 1.7, 2.9, 1.26, 0.9],
                   [0.5, 0.4, 0.3, 0.3, 3.1, 0.26, 0.1]])
    got = _check(lo, hi, 1.0)
    assert {tuple(p) for p in got} == {(0, 1), (0, 5), (0, 6), (1, 2), (1, 5), (1, 6), (2, 6), (3, 5), (5, 6)}


@pytest.mark.parametrize("n,span,size,H", [(1, 5.0, 1.0, 1.0), (2, 1.0, 1.0, 1.0), (300, 30.0, 2.0, 1.7),
                                           (3000, 200.0, 2.0, 2.5), (2500, 1000.0, 1.5, 0.8)])
def test_random_boxes(n, span, size, H):
    rng = np.random.default_rng(n)
    c = rng.uniform(0, span, (3, n))
    h = rng.uniform(0.05, 1.0, (3, n)) * size
    _check(c - h, c + h, H)


def test_crowded_cell_and_capacity():
    rng = np.random.default_rng(62)
    n = 700                                       # all boxes in one or two cells: long key segments
    c = rng.uniform(0.0, 1.0, (3, n))
    lo, hi = c - 0.01, c + 0.01
    full = _check(lo, hi, 2.0)
    assert len(full) == n * (n - 1) // 2
    part = host(S.collision_candidates(dev(lo), dev(hi), 2.0, capacity=1000)).T
    assert np.array_equal(part, full[:1000])


def test_empty_and_invalid_boxes():
    rng = np.random.default_rng(63)
    c = rng.uniform(0, 10, (3, 50))
    lo, hi = c - 0.6, c + 0.6
    lo[:, 7], hi[:, 7] = np.inf, -np.inf          # empty mesh
    lo[1, 11] = np.nan                             # NaN corner: no cells
    lo[:, 20], hi[:, 20] = 3.0, 2.0                # inverted
    got = _check(lo, hi, 1.1)
    assert not np.isin(got, [7, 11, 20]).any()
    assert S.collision_candidates(dev(np.zeros((3, 0))), dev(np.zeros((3, 0))), 1.0).shape == (2, 0)
    one = S.collision_candidates(dev(lo[:, :1]), dev(hi[:, :1]), 1.0)
    assert one.shape == (2, 0)


def test_multi_pass_sort():
    """Cell coordinates up to ~2^12 per axis: 36-bit keys, five radix passes,
    and more than one sort workgroup of entries."""
    rng = np.random.default_rng(64)
    n = 2500
    c = rng.uniform(0, 4000.0, (3, n))
    c[:, : n // 2] = rng.uniform(0, 40.0, (3, n // 2))      # a dense corner too
    h = rng.uniform(0.2, 2.0, (3, n))
    _check(c - h, c + h, 1.0)


def test_rejections():
    L = C.lib()
    ctx = S.context()
    rng = np.random.default_rng(65)
    c = rng.uniform(0, 10, (3, 40))
    lo, hi = dev(c - 0.5), dev(c + 0.5)
    size = ctypes.c_size_t()
    assert L.stokes_collision_workspace_size(ctx, 40, 10, ctypes.byref(size)) == C.OK
    ws = torch.empty(size.value, dtype=torch.uint8, device=device())
    out = torch.full((2, 100), -7, dtype=torch.int32, device=device())
    npairs, nent = ctypes.c_int64(-1), ctypes.c_int64(-1)

    def run(cell=1.0, max_entries=10, cap=100, wsb=size.value, lo_=lo):
        return L.stokes_collision_candidates(ctx, 40, ctypes.c_void_p(lo_.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                             cell, max_entries, ctypes.c_void_p(out.data_ptr()), cap,
                                             ctypes.byref(npairs), ctypes.byref(nent), ctypes.c_void_p(ws.data_ptr()),
                                             wsb, None)

    assert run(cell=0.0) == C.EINVAL and b"cell_size" in L.stokes_last_error()
    assert run(cell=float("nan")) == C.EINVAL
    assert run(cap=-1) == C.EINVAL
    assert run(wsb=size.value - 1) == C.EWORKSPACE
    rc = run()                                     # 40 boxes of side 1 on a unit grid need > 10 entries
    assert rc == C.EWORKSPACE and nent.value > 10 and b"max_entries" in L.stokes_last_error()
    big = dev(np.array([[0.0] * 40, [0.0] * 40, [0.0] * 40]))
    far = dev(np.array([[1e9] * 40, [0.5] * 40, [0.5] * 40]))
    rc = L.stokes_collision_candidates(ctx, 40, ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(far.data_ptr()),
                                       1.0, 10, ctypes.c_void_p(out.data_ptr()), 100, ctypes.byref(npairs), None,
                                       ctypes.c_void_p(ws.data_ptr()), size.value, None)
    assert rc == C.EUNSUPPORTED and b"2^21" in L.stokes_last_error()
    torch.cuda.synchronize()
    assert bool((out == -7).all())


def test_cells_and_wall_full_size():
    """The benchmark's workload: 3,840 cells in the vessel (their boxes over one
    time step) and the 4,096 wall patches, grid spacing = mean box diagonal."""
    cfg = W.make_config(4)
    cells = cfg["cells"]
    rng = np.random.default_rng(66)
    order = np.argsort(cells.group, kind="stable")
    pos = np.ascontiguousarray(cells.pos[:, order])
    grp = cells.group[order]
    from types import SimpleNamespace
    x1 = W.cells_after_step(rng, SimpleNamespace(pos=pos, group=grp))
    ofs = W.group_offsets(grp)
    wall = W.cylinder_wall()
    wofs = np.arange(0, wall.n + 1, wall.meta["points_per_patch"], dtype=np.int64)
    clo, chi = S.space_time_boxes(dev(ofs), dev(pos), dev(x1))
    wlo, whi = S.space_time_boxes(dev(wofs), dev(wall.pos))
    lo = torch.cat([clo, wlo], dim=1).contiguous()
    hi = torch.cat([chi, whi], dim=1).contiguous()
    rlo = np.concatenate(SP.space_time_boxes(pos, x1, ofs)[:1] + SP.space_time_boxes(wall.pos, None, wofs)[:1], axis=1)
    assert np.array_equal(host(lo), rlo)
    H = float(np.linalg.norm(host(hi) - host(lo), axis=0).mean())
    got = _check(host(lo), host(hi), H)
    assert len(got) > 1000
