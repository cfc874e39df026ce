"""CPU oracle of the spatial-hash candidate search -- test infrastructure only
(imported by ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark; never by the product package).

Sec. 4 (parallel collision handling), which reuses steps a-c of the parallel
closest-point search of Sec. 3.3: every mesh gets its space-time bounding box,
the smallest axis-aligned box holding the mesh at the start and at the end of
the time step (a patch does not move, so its box is its bounding box).  Boxes
are hashed on a grid of spacing H: the paper samples each box's volume at a
spacing below H and hashes the samples (Morton order of the grid cell); those
samples land in exactly the grid cells the box overlaps.  Meshes whose boxes
share a grid cell are collision candidates.

Readings:
  * The grid's origin is the lowest corner over all boxes; a coordinate x lies
    in cell floor((x - origin) / H), computed in float64 (the same division and
    floor on both sides, so the integer cells agree exactly).
  * Candidates are unordered pairs of distinct boxes (i < j) sharing at least
    one cell, each listed once.
  * A mesh with no points has the empty box lo = +inf, hi = -inf (the
    identities of min and max) and takes part in no pair; nor does any box
    with lo > hi on some axis.
The search here is brute force over all pairs: two boxes share a cell exactly
when their integer cell ranges overlap on all three axes.
"""
from __future__ import annotations

import numpy as np


def space_time_boxes(x0, x1, mesh_ofs, inflate=0.0):
    """(lo, hi), each (3, n_meshes): per mesh m, the min and max over its points
    mesh_ofs[m]..mesh_ofs[m+1] at both times (x1 may be None), moved out by
    `inflate` on every side."""
    x0 = np.asarray(x0, dtype=np.float64)
    n = len(mesh_ofs) - 1
    lo = np.empty((3, n))
    hi = np.empty((3, n))
    for m in range(n):
        a, b = mesh_ofs[m], mesh_ofs[m + 1]
        if b <= a:
            lo[:, m], hi[:, m] = np.inf, -np.inf
            continue
        pts = x0[:, a:b] if x1 is None else np.concatenate([x0[:, a:b], np.asarray(x1)[:, a:b]], axis=1)
        lo[:, m] = pts.min(axis=1) - inflate
        hi[:, m] = pts.max(axis=1) + inflate
    return lo, hi


def valid_boxes(lo, hi):
    """Boxes with lo <= hi on every axis."""
    return np.all(np.asarray(lo) <= np.asarray(hi), axis=0)


def cell_ranges(lo, hi, H, origin=None):
    """Integer cell ranges [clo, chi] (each (3, n), int64) of the valid boxes on
    the grid of spacing H whose origin is the lowest corner of the valid boxes
    (or `origin`); invalid boxes get the empty range clo = 1, chi = 0."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ok = valid_boxes(lo, hi)
    if origin is None:
        origin = lo[:, ok].min(axis=1) if ok.any() else np.zeros(3)
    o = np.asarray(origin, dtype=np.float64)[:, None]
    clo = np.ones(lo.shape, dtype=np.int64)
    chi = np.zeros(lo.shape, dtype=np.int64)
    clo[:, ok] = np.floor((lo[:, ok] - o) / H).astype(np.int64)
    chi[:, ok] = np.floor((hi[:, ok] - o) / H).astype(np.int64)
    return clo, chi


def collision_candidates(lo, hi, H):
    """All pairs (i, j), i < j, whose boxes share a grid cell, as an (n_pairs, 2)
    int64 array in lexicographic order."""
    clo, chi = cell_ranges(lo, hi, H)
    valid = valid_boxes(lo, hi)
    n = clo.shape[1]
    pairs = []
    for i in range(n):
        if not valid[i]:
            continue
        ok = valid[i + 1:].copy()
        for c in range(3):
            ok &= (clo[c, i + 1:] <= chi[c, i]) & (clo[c, i] <= chi[c, i + 1:])
        for j in np.nonzero(ok)[0]:
            pairs.append((i, i + 1 + j))
    return np.array(pairs, dtype=np.int64).reshape(-1, 2)


def morton3(cx, cy, cz, bits=21):
    """Morton code: bit k of x, y, z at positions 3k, 3k+1, 3k+2."""
    code = 0
    for k in range(bits):
        code |= ((int(cx) >> k) & 1) << (3 * k)
        code |= ((int(cy) >> k) & 1) << (3 * k + 1)
        code |= ((int(cz) >> k) & 1) << (3 * k + 2)
    return code
