"""Pins of the spatial-hash candidate oracle (Sec. 4, reusing steps a-c of
Sec. 3.3) against a hand-worked case and against the paper's own formulation,
independent of the oracle's range test.

  * hand-worked boxes (golden file), with a shared cell but no overlap and a
    box edge exactly on a cell boundary            -> the cell rule, the origin
  * hash-and-match: each box's cells enumerated, Morton keys collected in a
    dictionary, boxes with a common key paired      -> the range-overlap test, morton3
  * every overlapping pair of boxes is a candidate; every candidate pair is
    closer than H on each axis                      -> superset / locality
  * space-time boxes hold both positions of every point and touch them
"""
import os
from collections import defaultdict

import numpy as np

from oracle import spatial as SP

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "collision_boxes.txt")


def _golden():
    boxes, pairs = [], []
    for line in open(GOLDEN):
        t = line.split("#")[0].split()
        if not t:
            continue
        if t[0] == "box":
            boxes.append([float(v) for v in t[2:8]])
        elif t[0] == "pair":
            pairs.append((int(t[1]), int(t[2])))
    b = np.array(boxes).T
    return b[:3], b[3:], np.array(pairs, dtype=np.int64)


def test_hand_worked_boxes():
    lo, hi, want = _golden()
    got = SP.collision_candidates(lo, hi, 1.0)
    assert np.array_equal(got, want)


def _hash_and_match(lo, hi, H):
    clo, chi = SP.cell_ranges(lo, hi, H)
    table = defaultdict(list)
    for b in range(lo.shape[1]):
        for cx in range(clo[0, b], chi[0, b] + 1):
            for cy in range(clo[1, b], chi[1, b] + 1):
                for cz in range(clo[2, b], chi[2, b] + 1):
                    table[SP.morton3(cx, cy, cz)].append(b)
    pairs = set()
    for boxes in table.values():
        for i in range(len(boxes)):
            for j in range(i + 1, len(boxes)):
                pairs.add((min(boxes[i], boxes[j]), max(boxes[i], boxes[j])))
    return np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)


def _random_boxes(rng, n, span, size):
    c = rng.uniform(0, span, (3, n))
    h = rng.uniform(0.1, 1.0, (3, n)) * size
    return c - h, c + h


def test_hash_and_match_agrees():
    rng = np.random.default_rng(51)
    for n, span, size, H in ((60, 10.0, 1.0, 1.3), (200, 20.0, 2.0, 1.0), (120, 5.0, 0.3, 0.77)):
        lo, hi = _random_boxes(rng, n, span, size)
        assert np.array_equal(SP.collision_candidates(lo, hi, H), _hash_and_match(lo, hi, H))


def test_superset_and_locality():
    rng = np.random.default_rng(52)
    lo, hi = _random_boxes(rng, 300, 30.0, 2.0)
    H = 1.7
    got = {tuple(p) for p in SP.collision_candidates(lo, hi, H)}
    n = lo.shape[1]
    for i in range(n):
        for j in range(i + 1, n):
            overlap = all(lo[c, i] <= hi[c, j] and lo[c, j] <= hi[c, i] for c in range(3))
            if overlap:
                assert (i, j) in got
    for i, j in got:
        gap = np.maximum(lo[:, j] - hi[:, i], lo[:, i] - hi[:, j])
        assert np.all(gap < H)


def test_morton_interleaving():
    assert SP.morton3(1, 0, 0) == 1 and SP.morton3(0, 1, 0) == 2 and SP.morton3(0, 0, 1) == 4
    # x = 101, y = 011, z = 110 interleaved z2 y2 x2 z1 y1 x1 z0 y0 x0 = 1 0 1 1 1 0 0 1 1
    assert SP.morton3(0b101, 0b011, 0b110) == 0b101110011
    assert SP.morton3((1 << 21) - 1, (1 << 21) - 1, (1 << 21) - 1) == (1 << 63) - 1
    rng = np.random.default_rng(53)                  # monotone in each coordinate
    for _ in range(200):
        a = rng.integers(0, 1 << 20, 3)
        c = int(rng.integers(0, 3))
        b = a.copy()
        b[c] += 1
        assert SP.morton3(*b) > SP.morton3(*a)


def test_space_time_boxes():
    rng = np.random.default_rng(54)
    ofs = np.array([0, 5, 5, 12, 40])
    x0 = rng.standard_normal((3, 40))
    x1 = x0 + 0.3 * rng.standard_normal((3, 40))
    lo, hi = SP.space_time_boxes(x0, x1, ofs, inflate=0.0)
    for m in (0, 2, 3):
        pts = np.concatenate([x0[:, ofs[m]:ofs[m + 1]], x1[:, ofs[m]:ofs[m + 1]]], axis=1)
        assert np.all(pts >= lo[:, m:m + 1]) and np.all(pts <= hi[:, m:m + 1])
        assert np.all(np.any(pts == lo[:, m:m + 1], axis=1)) and np.all(np.any(pts == hi[:, m:m + 1], axis=1))
    assert np.all(lo[:, 1] == np.inf) and np.all(hi[:, 1] == -np.inf)     # the empty mesh
    lo2, hi2 = SP.space_time_boxes(x0, x1, ofs, inflate=0.25)
    keep = [0, 2, 3]
    assert np.array_equal(lo2[:, keep], lo[:, keep] - 0.25) and np.array_equal(hi2[:, keep], hi[:, keep] + 0.25)
    # an empty box is in no pair, even when it would cover everything
    lo3 = np.concatenate([lo2, [[5.0], [5.0], [5.0]]], axis=1)
    hi3 = np.concatenate([hi2, [[-5.0], [-5.0], [-5.0]]], axis=1)
    pairs = SP.collision_candidates(lo3, hi3, 0.5)
    assert not np.isin(pairs, [1, 4]).any()
    # an empty box next to a box whose range covers cells 0 and 1 (the empty range's values)
    lo4 = np.array([[0.0, 1.0], [0.0, 1.0], [0.0, 1.0]])
    hi4 = np.array([[1.5, 0.0], [1.5, 0.0], [1.5, 0.0]])
    assert SP.collision_candidates(lo4, hi4, 1.0).shape == (0, 2)
