"""Pair conservation of the mixed-precision split (direct and leaf-to-leaf).

The mixed paths take every pair once: in float32, as a float64 near pair
(distance within near_frac times the mesh spacing of the source's group), or
not at all (same group under the exclusion rule, or zero distance).  With the
library's test-only class record, each (target, source) pair's class is
compared with its exact float64 classification, on layouts that place pairs
at the near radius times (1 +- 1e-6).  Pairs within 1e-6 of the radius in
rho^2 may go either way (float32 rounding of the distance is below 5e-7
relative); the placed pairs sit at +-2e-6 and must fall on their own side.
"""
import numpy as np
import pytest
import torch

import paper_1909_11085_amd as S
from paper_1909_11085_amd import _capi as C
from paper_1909_11085_amd import workloads as W
from tests.gpu_util import dev, device, host

pytestmark = pytest.mark.gpu

NEAR_FRAC = 0.5
BAND = 1e-6
EDGE = 1e-6


def _unit(rng, n):
    u = rng.standard_normal((3, n))
    return u / np.linalg.norm(u, axis=0)


def _expected(x, gt, y, gs, h, excl):
    """Exact classes of all (target, source) pairs, the pairs inside the
    rounding band, and the placed pairs (ratio 1 +- 2e-6)."""
    d2 = np.zeros((x.shape[1], y.shape[1]))
    zero = np.ones(d2.shape, dtype=bool)
    for c in range(3):
        diff = x[c][:, None] - y[c][None, :]
        d2 += diff * diff
        zero &= diff == 0.0
    rn2 = (NEAR_FRAC * h[gs]) ** 2
    ratio = d2 / rn2[None, :] - 1.0
    skip = zero | (excl & (gt[:, None] == gs[None, :]))
    exp = np.where(skip, C.PAIR_SKIP, np.where(d2 <= rn2[None, :], C.PAIR_F64, C.PAIR_F32)).astype(np.int32)
    band = (np.abs(ratio) < BAND) & ~skip
    placed = (np.abs(np.abs(ratio) - 2 * EDGE) < 2e-7) & ~skip
    return exp, band, placed


def _check(cls, exp, band, placed, listed=None, what=""):
    got = host(cls)
    if listed is None:
        listed = np.ones(got.shape, dtype=bool)
    assert np.all(got[~listed] == 0), f"{what}: an unlisted pair was taken"
    g, e, b = got[listed], exp[listed], band[listed]
    once = np.isin(g, [C.PAIR_F32, C.PAIR_F64, C.PAIR_SKIP])
    assert once.all(), f"{what}: {int((~once).sum())} listed pairs not taken exactly once"
    ok = (g == e) | (b & (g != C.PAIR_SKIP))
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, f"{what}: {bad.size} pairs misclassified, e.g. got {g[bad[:5]]} want {e[bad[:5]]}"
    # per target: float32 + float64 + skipped = the listed sources
    per_t = np.stack([(got == c).sum(1) for c in (C.PAIR_F32, C.PAIR_F64, C.PAIR_SKIP)])
    assert np.array_equal(per_t.sum(0), listed.sum(1))
    n_placed = int((placed & listed).sum())
    print(f"{what}: {g.size} pairs: f32 {int((g == C.PAIR_F32).sum())}, f64 {int((g == C.PAIR_F64).sum())}, "
          f"skipped {int((g == C.PAIR_SKIP).sum())}; placed pairs at r_near(1 +- 1e-6): {n_placed}, "
          f"band pairs: {int(b.sum())}")
    return n_placed


# ---------------------------------------------------------------- direct
def _direct_layout(seed, ns=3000, nt=2400, n_groups=6, n_edge=800, n_dup=24):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-2.5, 2.5, (n_groups, 3))
    h = rng.uniform(0.3, 0.6, n_groups)
    gs = rng.integers(0, n_groups, ns).astype(np.int32)
    y = (centres[gs] + 0.7 * rng.standard_normal((ns, 3))).T.copy()
    gt = rng.integers(0, n_groups, nt).astype(np.int32)
    x = (centres[gt] + 0.7 * rng.standard_normal((nt, 3))).T.copy()
    # targets at r_near (1 +- 1e-6) from a source of another group
    k = rng.choice(ns, n_edge, replace=False)
    sign = np.where(np.arange(n_edge) % 2 == 0, 1.0, -1.0)
    x[:, :n_edge] = y[:, k] + _unit(rng, n_edge) * (NEAR_FRAC * h[gs[k]] * (1.0 + sign * EDGE))
    gt[:n_edge] = (gs[k] + 1 + rng.integers(0, n_groups - 1, n_edge)) % n_groups
    # targets on sources, half in the source's group
    j = rng.choice(ns, n_dup, replace=False)
    x[:, n_edge:n_edge + n_dup] = y[:, j]
    gt[n_edge:n_edge + n_dup] = np.where(np.arange(n_dup) % 2 == 0, gs[j], (gs[j] + 1) % n_groups)
    perm = rng.permutation(nt)
    x, gt = x[:, perm].copy(), gt[perm].copy()
    f = rng.standard_normal((3, ns))
    w = rng.uniform(0.1, 1.0, ns)
    return dict(x=x, gt=gt, y=y, gs=gs, h=h, f=f, w=w, n=_unit(rng, ns))


@pytest.mark.parametrize("kernel", ["sl", "dl"])
@pytest.mark.parametrize("excl", [True, False])
def test_direct_mixed_split(kernel, excl):
    print(f"case pair split direct {kernel} excl={excl}", flush=True)
    d = _direct_layout(141)
    nt, ns = d["x"].shape[1], d["y"].shape[1]
    cls = torch.zeros((nt, ns), dtype=torch.int32, device=device())
    kw = dict(src_group=dev(d["gs"]), trg_group=dev(d["gt"]), exclude_same_group=excl, precision="mixed",
              group_h=dev(d["h"]), near_frac=NEAR_FRAC)
    S.debug_pair_classes(cls)
    try:
        if kernel == "sl":
            S.sl(dev(d["y"]), dev(d["f"]), dev(d["w"]), dev(d["x"]), **kw)
        else:
            S.dl(dev(d["y"]), dev(d["f"]), dev(d["w"]), dev(d["n"]), dev(d["x"]), **kw)
    finally:
        S.debug_pair_classes(None)
    exp, band, placed = _expected(d["x"], d["gt"], d["y"], d["gs"], d["h"], excl)
    assert _check(cls, exp, band, placed, what=f"direct {kernel} excl={excl}") == 800


def test_pair_class_registration():
    """A registered array of other sizes makes a mixed call fail before any
    launch; float64 calls ignore it; None unregisters."""
    print("case pair class registration", flush=True)
    d = _direct_layout(142, ns=300, nt=200, n_edge=50, n_dup=4)
    cls = torch.zeros((7, 9), dtype=torch.int32, device=device())
    args = (dev(d["y"]), dev(d["f"]), dev(d["w"]), dev(d["x"]))
    kw = dict(src_group=dev(d["gs"]), trg_group=dev(d["gt"]), group_h=dev(d["h"]))
    S.debug_pair_classes(cls)
    try:
        with pytest.raises(C.StokesError) as e:
            S.sl(*args, precision="mixed", **kw)
        assert e.value.status == C.EINVAL
        S.sl(*args, precision="fp64", **kw)
    finally:
        S.debug_pair_classes(None)
    S.sl(*args, precision="mixed", **kw)
    assert int(host(cls).sum()) == 0


# ---------------------------------------------------------------- leaf-to-leaf
def _p2p_layout(seed, n_base=2600, n_edge=500, n_dup=16, n_groups=6):
    """A shared point set sorted into octree leaves; added points sit at
    r_near (1 +- 1e-6) from a base point of the partner group (groups 2k and
    2k+1 share their mesh spacing, so the pair is on the radius both ways)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 6.0, (n_groups, 3))
    h = np.repeat(rng.uniform(0.3, 0.6, n_groups // 2), 2)
    g = rng.integers(0, n_groups, n_base).astype(np.int32)
    y = (centres[g] + 0.7 * rng.standard_normal((n_base, 3))).T
    k = rng.choice(n_base, n_edge, replace=False)
    sign = np.where(np.arange(n_edge) % 2 == 0, 1.0, -1.0)
    pe = y[:, k] + _unit(rng, n_edge) * (NEAR_FRAC * h[g[k]] * (1.0 + sign * EDGE))
    j = rng.choice(n_base, n_dup, replace=False)
    gd = np.where(np.arange(n_dup) % 2 == 0, g[j], g[j] ^ 1).astype(np.int32)
    pos = np.concatenate([y, pe, y[:, j]], axis=1)
    grp = np.concatenate([g, g[k] ^ 1, gd]).astype(np.int32)
    lo = pos.min(1) - 1e-3
    side = float((pos.max(1) - lo).max()) + 1e-3
    tree = W.build_octree(pos, lo, side, max_leaf=48)
    p = tree.perm
    pos, grp = pos[:, p].copy(), grp[p].copy()
    n = pos.shape[1]
    f = rng.standard_normal((3, n))
    w = rng.uniform(0.1, 1.0, n)
    ofs, ul = W.nearest_leaf_lists(rng, tree, kmin=8, kmax=20)
    lof = tree.leaf_ofs
    listed = np.zeros((n, n), dtype=bool)
    for L in range(len(lof) - 1):
        for Ls in ul[ofs[L]:ofs[L + 1]]:
            listed[lof[L]:lof[L + 1], lof[Ls]:lof[Ls + 1]] = True
    return dict(pos=pos, g=grp, h=h, f=f, w=w, n=_unit(rng, n), tree=tree, ofs=ofs, ul=ul, listed=listed)


@pytest.mark.parametrize("kernel", ["sl", "dl"])
@pytest.mark.parametrize("excl", [True, False])
def test_p2p_mixed_split(kernel, excl):
    print(f"case pair split p2p {kernel} excl={excl}", flush=True)
    d = _p2p_layout(143)
    n = d["pos"].shape[1]
    plan = S.P2PPlan(d["tree"].leaf_ofs, d["tree"].leaf_ofs, d["ofs"], d["ul"], n, n)
    cls = torch.zeros((n, n), dtype=torch.int32, device=device())
    pos = dev(d["pos"])
    S.debug_pair_classes(cls)
    try:
        S.p2p_leaf(plan, pos, dev(d["f"]), dev(d["w"]), pos, kernel=kernel, nrm=dev(d["n"]),
                   src_group=dev(d["g"]), trg_group=dev(d["g"]), exclude_same_group=excl, precision="mixed",
                   group_h=dev(d["h"]), near_frac=NEAR_FRAC)
    finally:
        S.debug_pair_classes(None)
    exp, band, placed = _expected(d["pos"], d["g"], d["pos"], d["g"], d["h"], excl)
    n_placed = _check(cls, exp, band, placed, listed=d["listed"], what=f"p2p {kernel} excl={excl}")
    assert n_placed >= 500          # of the 1,000 placed ordered pairs, most are listed
