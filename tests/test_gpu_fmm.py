"""GPU parity of the kernel-independent FMM for the single- and double-layer
sums (Sec. 3.1, "Far evaluation") against the FMM oracle, and its accuracy
against the direct sum at sizes where only the GPU can run it.

The GPU and the oracle run the same algorithm; their operators are
pseudo-inverses from different SVD codes (one-sided Jacobi on the host here,
LAPACK in the oracle) with the same truncation.  Singular values kept near the
1e-10 cutoff are known only to about 1e-6 relative from either code, so the
two pseudo-inverses differ along those directions; the effect on the velocity
grows with the order.  The bars (1e-12 at order 2 up to 1e-6 from order 6 on)
are each far below the method's own error at that order; against the direct
sum the bar is that error.
"""
import ctypes
import itertools

import numpy as np
import pytest
import torch

import paper_1909_11085_amd as S
from oracle import fmm as F
from oracle import oracle as O
from paper_1909_11085_amd import _capi as C
from paper_1909_11085_amd import workloads as W
from tests.gpu_util import dev, device, host, rel_l2

pytestmark = pytest.mark.gpu

FMM_ERR = {4: 5e-3, 6: 3e-4}          # error against the direct sum (oracle pins: 1.5e-3, 6e-5)
# the double layer's far field converges more slowly (measured on the wall:
# 1.6e-2 at order 4, 1.0e-3 at order 6, ten times the single layer's)
FMM_ERR_DL = {4: 3e-2, 6: 2e-3}
# measured: 7.6e-15 (order 2), 1.0e-13 (3), below 1e-9 (4), 5.3e-10 (5), 5.5e-8 (6)
ORACLE_TOL = {2: 1e-12, 3: 1e-11, 4: 1e-9, 5: 1e-8, 6: 1e-6}
M2L_DENSE_FILL = 0.35     # the library's switch between the GEMM and pair sums


@pytest.fixture(scope="module")
def plans():
    return {p: S.FMMPlan(p) for p in (4, 6)}


def _cloud(seed, n, m):
    rng = np.random.default_rng(seed)
    src = rng.uniform(-1, 1, (3, n))
    src[:, : n // 3] = 0.2 * rng.standard_normal((3, n // 3)).clip(-4.9, 4.9)
    return src, rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), rng.uniform(-1, 1, (3, m))


@pytest.mark.parametrize("p", [4, 6])
def test_matches_oracle_fmm(plans, p):
    src, f, w, trg = _cloud(71, 1200, 300)
    got = host(S.fmm_sl(plans[p], dev(src), dev(f), dev(w), dev(trg), (0.0, 0.0, 0.0), 1.0001, 2, mu=1.3))
    ref = F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 2, p, mu=1.3)
    assert rel_l2(got, ref) < ORACLE_TOL[p], rel_l2(got, ref)
    direct = O.sl(src, f, w, trg, mu=1.3)
    assert rel_l2(got, direct) < FMM_ERR[p]


@pytest.mark.parametrize("p,D", [(4, 3), (4, 4), (6, 4)])
def test_accuracy_against_direct(plans, p, D):
    rng = np.random.default_rng(73 + D)
    n = 50_000
    src = rng.uniform(-2, 2, (3, n))
    src[:, : n // 2] = 0.4 * rng.standard_normal((3, n // 2)).clip(-4.9, 4.9)
    f, w = rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n)
    trg = src[:, ::7].copy()
    trg[:, ::2] += 0.01                                  # some targets on sources, some off
    S_, F_, W_, T_ = dev(src), dev(f), dev(w), dev(trg)
    got = host(S.fmm_sl(plans[p], S_, F_, W_, T_, (0.0, 0.0, 0.0), 2.0001, D))
    ref = host(S.sl(S_, F_, W_, T_))
    assert rel_l2(got, ref) < FMM_ERR[p], rel_l2(got, ref)


def test_depth_seven(plans):
    """The deepest tree (2,097,152 leaves): 300k clustered points, order 4, a
    seeded sample of targets against the direct sum."""
    rng = np.random.default_rng(83)
    n = 300_000
    src = rng.uniform(-2, 2, (3, n))
    src[:, : n // 2] = 0.4 * rng.standard_normal((3, n // 2)).clip(-4.9, 4.9)
    f, w = rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n)
    S_, F_, W_ = dev(src), dev(f), dev(w)
    got = S.fmm_sl(plans[4], S_, F_, W_, S_, (0.0, 0.0, 0.0), 2.0001, 7)
    pick = W.subset(np.random.default_rng(84), n, 2000)
    ref = host(S.sl(S_, F_, W_, dev(src[:, pick])))
    err = rel_l2(host(got)[:, pick], ref)
    assert err < FMM_ERR[4], err


def test_cells_workload_sampled(plans):
    """The 3,840 cells in the vessel (2,088,960 points), depth 6: all targets in
    one launch, a seeded sample against the direct sum (no pair rule)."""
    cfg = W.make_config(4)
    c = cfg["cells"]
    lo, hi = c.pos.min(axis=1), c.pos.max(axis=1)
    ctr, R = 0.5 * (lo + hi), 0.5 * float((hi - lo).max()) * 1.0001
    pos, f, w = dev(c.pos), dev(cfg["f"]), dev(c.weight)
    got = S.fmm_sl(plans[4], pos, f, w, pos, tuple(ctr), R, 6)
    pick = W.subset(np.random.default_rng(74), c.n, 2000)
    ref = host(S.sl(pos, f, w, dev(c.pos[:, pick])))
    err = rel_l2(host(got)[:, pick], ref)
    assert err < FMM_ERR[4], err
    assert bool(torch.isfinite(got).all())


def _normals(seed, n):
    nrm = np.random.default_rng(seed).standard_normal((3, n))
    return nrm / np.linalg.norm(nrm, axis=0)


@pytest.mark.parametrize("p", [4, 6])
def test_dl_matches_oracle_fmm(plans, p):
    src, f, w, trg = _cloud(77, 1000, 250)
    nrm = _normals(78, 1000)
    got = host(S.fmm_dl(plans[p], dev(src), dev(f), dev(w), dev(nrm), dev(trg), (0.0, 0.0, 0.0), 1.0001, 2))
    ref = F.fmm_dl(src, f, w, nrm, trg, np.zeros(3), 1.0001, 2, p)
    assert rel_l2(got, ref) < ORACLE_TOL[p], rel_l2(got, ref)
    assert rel_l2(got, O.dl(src, f, w, nrm, trg)) < FMM_ERR_DL[p]


@pytest.mark.parametrize("p", [4, 6])
def test_dl_accuracy_against_direct(plans, p):
    rng = np.random.default_rng(79)
    n = 40_000
    src = rng.uniform(-2, 2, (3, n))
    src[:, : n // 2] = 0.4 * rng.standard_normal((3, n // 2)).clip(-4.9, 4.9)
    f, w, nrm = rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), _normals(80, n)
    trg = rng.uniform(-2, 2, (3, 5000))
    args = [dev(src), dev(f), dev(w), dev(nrm), dev(trg)]
    got = host(S.fmm_dl(plans[p], *args, (0.0, 0.0, 0.0), 2.0001, 4))
    ref = host(S.dl(*args))
    assert rel_l2(got, ref) < FMM_ERR_DL[p], rel_l2(got, ref)


def test_dl_wall_onto_cells_sampled(plans):
    """The vessel wall's double layer (1,048,576 nodes) at the 522,240 points
    of 960 cells, depth 6, order 6: all targets in one launch, a sample against
    the direct sum."""
    cfg = W.make_config(5)
    wall, cells = cfg["wall"], cfg["cells"]
    lo = np.minimum(wall.pos.min(axis=1), cells.pos.min(axis=1))
    hi = np.maximum(wall.pos.max(axis=1), cells.pos.max(axis=1))
    ctr, R = 0.5 * (lo + hi), 0.5 * float((hi - lo).max()) * 1.0001
    args = [dev(wall.pos), dev(cfg["phi"]), dev(wall.weight), dev(wall.normal)]
    got = S.fmm_dl(plans[6], *args, dev(cells.pos), tuple(ctr), R, 6)
    pick = W.subset(np.random.default_rng(81), cells.n, 2000)
    ref = host(S.dl(*args, dev(cells.pos[:, pick])))
    err = rel_l2(host(got)[:, pick], ref)
    assert err < FMM_ERR_DL[6], err


@pytest.mark.parametrize("p", [2, 3, 5])
def test_other_orders_match_oracle(p):
    """Orders 2, 3 and 5 (the other tile shapes of the M2L and pseudo-inverse
    GEMMs) against the oracle FMM, single and double layer."""
    plan = S.FMMPlan(p)
    src, f, w, trg = _cloud(77, 900, 250)
    got = host(S.fmm_sl(plan, dev(src), dev(f), dev(w), dev(trg), (0.0, 0.0, 0.0), 1.0001, 2, mu=1.3))
    ref = F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 2, p, mu=1.3)
    assert rel_l2(got, ref) < ORACLE_TOL[p], rel_l2(got, ref)
    nrm = _normals(78, 900)
    got = host(S.fmm_dl(plan, dev(src), dev(f), dev(w), dev(nrm), dev(trg), (0.0, 0.0, 0.0), 1.0001, 2))
    ref = F.fmm_dl(src, f, w, nrm, trg, np.zeros(3), 1.0001, 2, p)
    assert rel_l2(got, ref) < ORACLE_TOL[p], rel_l2(got, ref)


def _two_clusters(seed, n=400, m=60):
    rng = np.random.default_rng(seed)
    src = np.concatenate([rng.uniform(-0.95, -0.55, (3, n // 2)), rng.uniform(0.3, 0.9, (3, n // 2))], axis=1)
    trg = np.concatenate([rng.uniform(-0.95, -0.55, (3, m // 2)), rng.uniform(0.3, 0.9, (3, m // 2))], axis=1)
    trg[:, ::2] = rng.uniform(-1, 1, (3, m // 2))
    return src, rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), trg


# orders 7 .. 10 (the GEMM rows cut into 2, 2, 3 and 4 row groups, 4 .. 8
# check points per lane): against the oracle FMM (measured 9e-9 .. 5e-8) and
# the direct sum (measured 4.3e-7, 1.6e-7, 2.3e-8, 9.2e-9 on this cloud)
HIGH_ORDER_DIRECT = {7: 3e-6, 8: 1e-6, 9: 2e-7, 10: 1e-7}


@pytest.mark.parametrize("p", [7, 8, 9, 10])
def test_high_orders_match_oracle(p):
    print(f"case fmm order {p} vs oracle", flush=True)
    plan = S.FMMPlan(p)
    src, f, w, trg = _two_clusters(3)
    got = host(S.fmm_sl(plan, dev(src), dev(f), dev(w), dev(trg), (0.0, 0.0, 0.0), 1.0001, 2))
    ref = F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 2, p)
    assert rel_l2(got, ref) < 1e-6, rel_l2(got, ref)
    assert rel_l2(got, O.sl(src, f, w, trg)) < HIGH_ORDER_DIRECT[p], rel_l2(got, O.sl(src, f, w, trg))


def test_order_ten_reaches_the_mixed_bar():
    """Order 10 against the direct sums on 16 cells (2,304 points) at depths 3
    and 4, single and double layer: within 1e-6 (measured 1.1e-7 .. 3.9e-7),
    the bar of the mixed-precision direct sum."""
    print("case fmm order 10 cells", flush=True)
    rng = np.random.default_rng(5)
    c = W.place_cells(rng, 16, ("box", 20.0), order=8)
    f = rng.standard_normal((3, c.n))
    lo, hi = c.pos.min(1), c.pos.max(1)
    ctr, R = 0.5 * (lo + hi), 0.5 * float((hi - lo).max()) * 1.0001
    ref = O.sl(c.pos, f, c.weight, c.pos)
    refd = O.dl(c.pos, f, c.weight, c.normal, c.pos)
    plan = S.FMMPlan(10)
    pos, F_, W_ = dev(c.pos), dev(f), dev(c.weight)
    for D in (3, 4):
        u = host(S.fmm_sl(plan, pos, F_, W_, pos, tuple(ctr), R, D))
        ud = host(S.fmm_dl(plan, pos, F_, W_, dev(c.normal), pos, tuple(ctr), R, D))
        assert rel_l2(u, ref) < 1e-6, (D, rel_l2(u, ref))
        assert rel_l2(ud, refd) < 1e-6, (D, rel_l2(ud, refd))


def _il_fill(src, trg, R, l):
    """Fraction of the 189 interaction-list offsets of the target boxes of
    level l (cube centred at 0, half-width R) that hold sources."""
    n = 2 ** l
    box = lambda x: np.clip(np.floor((x + R) / (2 * R / n)).astype(int), 0, n - 1)
    sb = set(map(tuple, box(src).T))
    tb = set(map(tuple, box(trg).T))
    hits = 0
    for b in map(np.array, tb):
        for d in itertools.product((-1, 0, 1), repeat=3):
            pn = b // 2 + np.array(d)
            if np.any(pn < 0) or np.any(pn >= n // 2):
                continue
            for o in itertools.product((0, 1), repeat=3):
                a = 2 * pn + np.array(o)
                if np.max(np.abs(a - b)) > 1 and tuple(a) in sb:
                    hits += 1
    return hits / (len(tb) * 189)


@pytest.mark.parametrize("layout", ["filled", "separated"])
def test_m2l_paths_match_oracle(plans, layout):
    """Sources filling the cube give dense interaction lists (the M2L GEMM);
    sources in one corner and targets in the opposite one give sparse lists
    (M2L as pair sums).  Both against the oracle FMM at depth 3."""
    rng = np.random.default_rng(91 if layout == "filled" else 92)
    if layout == "filled":
        src, trg = rng.uniform(-1, 1, (3, 3000)), rng.uniform(-0.3, 0.3, (3, 200))
    else:
        src, trg = rng.uniform(-1, -0.5, (3, 3000)), rng.uniform(0.5, 1, (3, 200))
    # level 2 offers at most 37 of the 189 offsets, so it always runs as pair sums
    fills = [_il_fill(src, trg, 1.0001, l) for l in (2, 3)]
    if layout == "filled":
        assert fills[1] >= M2L_DENSE_FILL, fills
    else:
        assert max(fills) < M2L_DENSE_FILL and fills[0] > 0, fills
    f, w = rng.standard_normal((3, 3000)), rng.uniform(0.5, 1.0, 3000)
    got = host(S.fmm_sl(plans[4], dev(src), dev(f), dev(w), dev(trg), (0.0, 0.0, 0.0), 1.0001, 3))
    ref = F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 3, 4)
    assert rel_l2(got, ref) < ORACLE_TOL[4], rel_l2(got, ref)


@pytest.mark.parametrize("layout", ["filled", "separated"])
def test_dl_m2l_paths_match_oracle(plans, layout):
    """The double layer on both M2L paths at depth 3 against the oracle FMM:
    the point-source flux of each box rides through M2M and both forms of
    M2L.  Densities along the normals, so every box carries a net flux."""
    rng = np.random.default_rng(93 if layout == "filled" else 94)
    if layout == "filled":
        src, trg = rng.uniform(-1, 1, (3, 3000)), rng.uniform(-0.3, 0.3, (3, 200))
    else:
        src, trg = rng.uniform(-1, -0.5, (3, 3000)), rng.uniform(0.5, 1, (3, 200))
    fills = [_il_fill(src, trg, 1.0001, l) for l in (2, 3)]
    if layout == "filled":
        assert fills[1] >= M2L_DENSE_FILL, fills
    else:
        assert max(fills) < M2L_DENSE_FILL and fills[0] > 0, fills
    nrm = _normals(95, 3000)
    phi = nrm * rng.uniform(0.5, 1.5, 3000)
    w = rng.uniform(0.5, 1.0, 3000)
    got = host(S.fmm_dl(plans[4], dev(src), dev(phi), dev(w), dev(nrm), dev(trg), (0.0, 0.0, 0.0), 1.0001, 3))
    ref = F.fmm_dl(src, phi, w, nrm, trg, np.zeros(3), 1.0001, 3, 4)
    assert rel_l2(got, ref) < ORACLE_TOL[4], rel_l2(got, ref)
    assert rel_l2(got, O.dl(src, phi, w, nrm, trg)) < FMM_ERR_DL[4]


def _deep_inputs(kernel):
    from tests.test_fmm_pins import _deep_cloud
    src, f, w, trg = _deep_cloud(111)
    nrm = None
    if kernel == "dl":
        rng = np.random.default_rng(112)
        nrm = rng.standard_normal(src.shape)
        nrm /= np.linalg.norm(nrm, axis=0)
        f = nrm * rng.uniform(0.5, 1.5, src.shape[1])
    return src, f, w, nrm, trg


@pytest.mark.parametrize("kernel", ["sl", "dl"])
@pytest.mark.parametrize("D", [3, 4])
def test_deep_tree_matches_oracle(plans, kernel, D):
    """Depths 3 and 4 against the oracle FMM (the layout of its deep-tree
    pins: M2M, M2L and L2L at every level, targets on sources), in float64
    and with float32 near-field pairs."""
    src, f, w, nrm, trg = _deep_inputs(kernel)
    if kernel == "sl":
        ref = F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, D, 4, mu=0.8)
        run = lambda prec: host(S.fmm_sl(plans[4], dev(src), dev(f), dev(w), dev(trg), (0.0, 0.0, 0.0),
                                         1.0001, D, mu=0.8, precision=prec))
    else:
        ref = F.fmm_dl(src, f, w, nrm, trg, np.zeros(3), 1.0001, D, 4)
        run = lambda prec: host(S.fmm_dl(plans[4], dev(src), dev(f), dev(w), dev(nrm), dev(trg),
                                         (0.0, 0.0, 0.0), 1.0001, D, precision=prec))
    got = run("fp64")
    e64 = rel_l2(got, ref)
    assert e64 < ORACLE_TOL[4], e64
    mixed = run("mixed")
    e32 = rel_l2(mixed, ref)
    assert np.all(np.isfinite(mixed)) and e32 < MIXED_VS_FP64[kernel], e32
    print(f"deep tree {kernel} D={D}: fp64 {e64:.2e}, mixed {e32:.2e} vs the oracle FMM")


# float32 near-field pairs against the float64 FMM.  An offset of size d from
# the leaf centre carries 2^-24 d, so a pair at distance rho errs by about
# 6e-8 d / rho relative, times the kernel's degree (1 for the single layer, 5
# for the double layer's r^3 / rho^5).  This cloud puts targets 0.01 from
# sources in leaves 0.25 wide: measured 5.3e-6 for the double layer.
MIXED_VS_FP64 = {"sl": 1e-6, "dl": 2e-5}


def test_fmm_minus_self_cells_is_the_excluded_sum(plans):
    """The paper sums every pair by the FMM and replaces each cell's own terms
    by its singular quadrature.  Without that replacement: the FMM over all
    pairs minus each cell's sum onto itself (the leaf P2P with every cell a
    leaf whose list is itself) equals the direct sum with the same-cell rule,
    within the FMM's error (taken against the smaller excluded sum).  128
    cells, 69,632 points."""
    cfg = W.make_config(3)
    c = cfg["cells"]
    g = c.group
    assert np.all(np.diff(g) >= 0)                       # points come cell by cell
    n_cells = int(g.max()) + 1
    ofs = np.searchsorted(g, np.arange(n_cells + 1)).astype(np.int64)
    own = S.P2PPlan(ofs, ofs, np.arange(n_cells + 1, dtype=np.int64), np.arange(n_cells, dtype=np.int32), c.n, c.n)
    pos, f, w = dev(c.pos), dev(cfg["f"]), dev(c.weight)
    lo, hi = c.pos.min(axis=1), c.pos.max(axis=1)
    ctr, R = 0.5 * (lo + hi), 0.5 * float((hi - lo).max()) * 1.0001
    u = S.fmm_sl(plans[6], pos, f, w, pos, tuple(ctr), R, 4)
    u -= S.p2p_leaf(own, pos, f, w, pos, kernel="sl")
    grp = torch.as_tensor(g, dtype=torch.int32, device=device())
    ref = host(S.sl(pos, f, w, pos, src_group=grp, trg_group=grp, exclude_same_group=True))
    assert rel_l2(host(u), ref) < 3 * FMM_ERR[6], rel_l2(host(u), ref)
    # the FMM's own same-group rule is that composition: the points already
    # come group by group, so its stable sort keeps them in place
    ruled = S.fmm_sl(plans[6], pos, f, w, pos, tuple(ctr), R, 4, src_group=grp, trg_group=grp, n_groups=n_cells)
    assert torch.equal(ruled, u)


def test_same_group_rule_on_shuffled_points(plans):
    """The same-group rule with the points in random order (groups
    interleaved), single and double layer, against the direct sums with the
    rule; an id outside [0, n_groups) turns the output into NaN."""
    print("case fmm same-group rule, shuffled", flush=True)
    rng = np.random.default_rng(77)
    cfg = W.make_config(1)
    c = cfg["cells"]
    perm = rng.permutation(c.n)
    pos, f, w = dev(c.pos[:, perm]), dev(cfg["f"][:, perm]), dev(c.weight[perm])
    nrm = dev(c.normal[:, perm])
    grp = torch.as_tensor(c.group[perm], dtype=torch.int32, device=device())
    lo, hi = c.pos.min(axis=1), c.pos.max(axis=1)
    ctr, R = tuple(0.5 * (lo + hi)), 0.5 * float((hi - lo).max()) * 1.0001
    u = host(S.fmm_sl(plans[6], pos, f, w, pos, ctr, R, 3, src_group=grp, trg_group=grp))
    ref = host(S.sl(pos, f, w, pos, src_group=grp, trg_group=grp, exclude_same_group=True))
    assert rel_l2(u, ref) < 3 * FMM_ERR[6], rel_l2(u, ref)
    ud = host(S.fmm_dl(plans[6], pos, f, w, nrm, pos, ctr, R, 3, src_group=grp, trg_group=grp))
    refd = host(S.dl(pos, f, w, nrm, pos, src_group=grp, trg_group=grp, exclude_same_group=True))
    assert rel_l2(ud, refd) < 3 * FMM_ERR_DL[6], rel_l2(ud, refd)
    n_groups = int(c.group.max()) + 1
    bad = grp.clone()
    bad[5] = n_groups
    out = host(S.fmm_sl(plans[6], pos, f, w, pos, ctr, R, 3, src_group=bad, trg_group=grp, n_groups=n_groups))
    assert np.all(np.isnan(out))


@pytest.mark.parametrize("kernel", ["sl", "dl"])
def test_mixed_near_field(plans, kernel):
    """precision="mixed" (float32 near-field pairs) against the float64 FMM on
    the same tree, and against the direct sum within the FMM's error.  The
    cloud has coincident sources and targets (the zero-distance mask in
    float32)."""
    rng = np.random.default_rng(85)
    n = 60_000
    src = rng.uniform(-2, 2, (3, n))
    src[:, : n // 2] = 0.4 * rng.standard_normal((3, n // 2)).clip(-4.9, 4.9)
    f, w, nrm = rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), _normals(86, n)
    trg = src[:, ::5].copy()
    trg[:, ::2] += 0.01
    S_, F_, W_, N_, T_ = dev(src), dev(f), dev(w), dev(nrm), dev(trg)
    if kernel == "sl":
        run = lambda prec: host(S.fmm_sl(plans[4], S_, F_, W_, T_, (0.0, 0.0, 0.0), 2.0001, 4, precision=prec))
        ref = host(S.sl(S_, F_, W_, T_))
        bar = FMM_ERR[4]
    else:
        run = lambda prec: host(S.fmm_dl(plans[4], S_, F_, W_, N_, T_, (0.0, 0.0, 0.0), 2.0001, 4, precision=prec))
        ref = host(S.dl(S_, F_, W_, N_, T_))
        bar = FMM_ERR_DL[4]
    mixed, fp64 = run("mixed"), run("fp64")
    assert np.all(np.isfinite(mixed))
    assert rel_l2(mixed, fp64) < MIXED_VS_FP64[kernel], rel_l2(mixed, fp64)
    assert rel_l2(mixed, ref) < bar


def test_graph_capture_replays(plans):
    """An evaluation runs on one stream with no host round trip and no memset,
    so it can be captured in a HIP graph.  Three replays, with eager work and
    synchronisations between them, each bitwise equal to the eager result."""
    src, f, w, trg = _cloud(87, 20_000, 5_000)
    S_, F_, W_, T_ = dev(src), dev(f), dev(w), dev(trg)
    args = (plans[4], S_, F_, W_, T_, (0.0, 0.0, 0.0), 1.0001, 4)
    eager = host(S.fmm_sl(*args))
    out = torch.empty((3, trg.shape[1]), dtype=torch.float64, device=device())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        S.fmm_sl(*args, out=out)                        # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        S.fmm_sl(*args, out=out)
    for k in range(3):
        out.fill_(float(k + 7))
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), eager), k
        assert np.array_equal(host(S.fmm_sl(*args)), eager)   # eager work between the replays
        torch.cuda.synchronize()


def test_graph_capture_same_cell_mixed(plans):
    """The same-cell rule (group sort, leaf-to-leaf correction) and the mixed
    near field inside a captured graph: three replays, each bitwise equal to
    the eager result; the rule against the direct sum with the rule."""
    print("case fmm graph capture, same-cell rule, mixed", flush=True)
    cfg = W.make_config(1)
    c = cfg["cells"]
    pos, f, w = dev(c.pos), dev(cfg["f"]), dev(c.weight)
    grp = torch.as_tensor(c.group, dtype=torch.int32, device=device())
    ng = int(c.group.max()) + 1
    lo, hi = c.pos.min(axis=1), c.pos.max(axis=1)
    args = (plans[4], pos, f, w, pos, tuple(0.5 * (lo + hi)), 0.5 * float((hi - lo).max()) * 1.0001, 3)
    kw = dict(src_group=grp, trg_group=grp, n_groups=ng, precision="mixed")
    eager = host(S.fmm_sl(*args, **kw))
    ref = host(S.sl(pos, f, w, pos, src_group=grp, trg_group=grp, exclude_same_group=True))
    assert rel_l2(eager, ref) < 3 * FMM_ERR[4], rel_l2(eager, ref)
    out = torch.empty_like(pos)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        S.fmm_sl(*args, out=out, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        S.fmm_sl(*args, out=out, **kw)
    for k in range(3):
        out.fill_(float(k + 3))
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), eager), k
        assert np.array_equal(host(S.fmm_sl(*args, **kw)), eager)
        torch.cuda.synchronize()


def test_edge_cases(plans):
    src, f, w, trg = _cloud(75, 500, 100)
    P = plans[4]
    z = S.fmm_sl(P, dev(np.zeros((3, 0))), dev(np.zeros((3, 0))), dev(np.zeros(0)), dev(trg), (0, 0, 0), 1.0001, 2)
    assert not bool(z.abs().max())                       # no sources: zeros
    e = S.fmm_sl(P, dev(src), dev(f), dev(w), dev(np.zeros((3, 0))), (0, 0, 0), 1.0001, 3)
    assert tuple(e.shape) == (3, 0)                      # no targets: nothing to do
    base = torch.full((3, 100), 0.5, dtype=torch.float64, device=device())
    S.fmm_sl(P, dev(src), dev(f), dev(w), dev(trg), (0, 0, 0), 1.0001, 3, out=base, accumulate=True)
    one = host(S.fmm_sl(P, dev(src), dev(f), dev(w), dev(trg), (0, 0, 0), 1.0001, 3))
    assert np.array_equal(host(base), one + 0.5) or rel_l2(host(base), one + 0.5) < 1e-15
    # points a little outside the cube go to the boundary leaves and stay finite
    out = host(S.fmm_sl(P, dev(src * 1.05), dev(f), dev(w), dev(trg), (0, 0, 0), 1.0, 3))
    assert np.all(np.isfinite(out))
    # identical results from one run to the next
    again = host(S.fmm_sl(P, dev(src), dev(f), dev(w), dev(trg), (0, 0, 0), 1.0001, 3))
    assert np.array_equal(again, one)


def test_rejections(plans):
    L = C.lib()
    ctx = S.context()
    h = ctypes.c_void_p()
    assert L.stokes_fmm_plan_create(ctx, 1, ctypes.byref(h)) == C.EINVAL
    assert L.stokes_fmm_plan_create(ctx, 11, ctypes.byref(h)) == C.EINVAL
    P = plans[4].handle
    size = ctypes.c_size_t()
    assert L.stokes_fmm_workspace_size(ctx, P, 10, 10, 1, None, ctypes.byref(size)) == C.EINVAL
    assert L.stokes_fmm_workspace_size(ctx, P, 10, 10, 8, None, ctypes.byref(size)) == C.EINVAL
    g = torch.zeros(10, dtype=torch.int32, device=device())
    no_groups = C.Exclusion(C.EXCL_SAME_GROUP, g.data_ptr(), g.data_ptr(), None, 0, 0.0)
    assert L.stokes_fmm_workspace_size(ctx, P, 10, 10, 2, ctypes.byref(no_groups), ctypes.byref(size)) == C.EINVAL
    assert L.stokes_fmm_workspace_size(ctx, P, 10, 10, 2, None, ctypes.byref(size)) == C.OK
    ws = torch.empty(size.value, dtype=torch.uint8, device=device())
    x = dev(np.random.default_rng(76).uniform(-1, 1, (3, 10)))
    f, w = dev(np.ones((3, 10))), dev(np.ones(10))
    out = torch.full((3, 10), 9.0, dtype=torch.float64, device=device())
    c = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())

    def run(mu=1.0, centre=c, hw=1.0, opts=None, wsb=size.value, excl=None):
        return L.stokes_fmm_sl_eval(ctx, P, 10, vp(x), vp(f), vp(w), 10, vp(x), mu, centre, hw, 2,
                                    ctypes.byref(excl) if excl else None, ctypes.byref(opts) if opts else None,
                                    vp(out), vp(ws), wsb, None)

    assert run(mu=0.0) == C.EINVAL
    assert run(centre=None) == C.EINVAL
    assert run(hw=-1.0) == C.EINVAL
    assert run(opts=C.Opts(7, 0)) == C.EINVAL
    assert run(wsb=size.value - 1) == C.EWORKSPACE
    assert run(excl=no_groups) == C.EINVAL                              # the rule needs n_groups > 0
    one_group = C.Exclusion(C.EXCL_SAME_GROUP, g.data_ptr(), g.data_ptr(), None, 1, 0.0)
    assert run(excl=one_group) == C.EWORKSPACE                          # its correction needs more room
    torch.cuda.synchronize()
    assert bool((out == 9.0).all())
    assert run() == C.OK
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
