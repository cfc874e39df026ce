"""Pins of the kernel-independent FMM oracle (Sec. 3.1, "Far evaluation")
against the direct sum and against facts of its own construction, independent
of the FMM code.

  * the FMM velocity equals the direct sum within the method's error, which
    falls with the surface order p (measured 1.5e-3 at p = 4, 6e-5 at p = 6)
                                              -> interaction lists, passes
  * the pseudo-inverses satisfy K X K = K and X K X = X
                                              -> the check-to-equivalent solve
  * an upward equivalent density reproduces its box's field far away
                                              -> surfaces, radii, scaling
  * at depths 3 and 4 (M2M from the leaves up, L2L down to the leaves, and,
    for the double layer, each box's point-source flux carried up through
    M2M) the velocity still equals the direct sum within the method's error,
    on a double-layer cloud whose every box has a net flux (density along the
    normal)                                   -> the multi-level passes
"""
import numpy as np
import pytest

from oracle import fmm as F
from oracle import oracle as O


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cloud(seed, n, m):
    rng = np.random.default_rng(seed)
    src = rng.uniform(-1, 1, (3, n))
    src[:, : n // 3] = 0.2 * rng.standard_normal((3, n // 3)).clip(-4.9, 4.9)     # a cluster
    return src, rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), rng.uniform(-1, 1, (3, m))


def test_fmm_matches_direct_sum():
    src, f, w, trg = _cloud(71, 1200, 300)
    ref = O.sl(src, f, w, trg, mu=1.3)
    e4 = rel(F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 2, 4, mu=1.3), ref)
    e6 = rel(F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 2, 6, mu=1.3), ref)
    assert e4 < 5e-3 and e6 < 3e-4 and e6 < e4 / 10, (e4, e6)
    # targets at the sources (zero-distance pairs skipped on both sides)
    e = rel(F.fmm_sl(src, f, w, src[:, :200], np.zeros(3), 1.0001, 2, 6), O.sl(src, f, w, src[:, :200]))
    assert e < 3e-4, e


def test_dl_fmm_matches_direct_sum():
    src, f, w, trg = _cloud(74, 1000, 250)
    rng = np.random.default_rng(75)
    nrm = rng.standard_normal((3, 1000))
    nrm /= np.linalg.norm(nrm, axis=0)
    ref = O.dl(src, f, w, nrm, trg)
    e4 = rel(F.fmm_dl(src, f, w, nrm, trg, np.zeros(3), 1.0001, 2, 4), ref)
    e6 = rel(F.fmm_dl(src, f, w, nrm, trg, np.zeros(3), 1.0001, 2, 6), ref)
    assert e4 < 5e-3 and e6 < 3e-4 and e6 < e4 / 10, (e4, e6)
    # the double-layer kernel matrix itself against the direct oracle
    K = F.dl_matrix(trg[:, :5].T, src.T, nrm.T)
    q = (w[None, :] * f).T.reshape(-1)
    assert rel((K @ q).reshape(5, 3).T, O.dl(src, f, w, nrm, trg[:, :5])) < 1e-13


def test_pseudo_inverses():
    s, up, down = F.operators(4, mu=0.7)
    for a_c, a_e, X in ((F.ALPHA_UC, F.ALPHA_UE, up), (F.ALPHA_DC, F.ALPHA_DE, down)):
        K = F.kernel_matrix(a_c * s, a_e * s, mu=0.7)
        assert np.linalg.norm(K @ X @ K - K) <= 1e-10 * np.linalg.norm(K)
        assert np.linalg.norm(X @ K @ X - X) <= 1e-6 * np.linalg.norm(X)


def test_equivalent_density_reproduces_far_field():
    rng = np.random.default_rng(72)
    s, up, _ = F.operators(6)
    h = 0.37
    ctr = np.array([0.3, -0.2, 0.5])
    y = ctr[:, None] + h * rng.uniform(-1, 1, (3, 40))
    q = rng.standard_normal((40, 3))
    chk = ctr + F.ALPHA_UC * h * s
    dens = (h * up @ (F.kernel_matrix(chk, y.T) @ q.reshape(-1))).reshape(-1, 3)
    d = rng.standard_normal((3, 50))
    far = ctr[:, None] + 4.0 * h * d / np.abs(d).max(axis=0)       # on the cube of half-width 4h
    got = F.kernel_matrix(far.T, ctr + F.ALPHA_UE * h * s) @ dens.reshape(-1)
    ref = F.kernel_matrix(far.T, y.T) @ q.reshape(-1)
    assert rel(got, ref) < 1e-4                                     # measured 3.8e-5


def _deep_cloud(seed, n=1000, m=150):
    """Sources over the whole cube (a third in a cluster) and targets inside
    one level-3 box, split over two level-4 leaves, some of them on sources.
    Every level from 2 down has interaction lists with sources, so M2M, M2L
    and L2L all run; the few target boxes keep the oracle's M2L cheap."""
    rng = np.random.default_rng(seed)
    src = rng.uniform(-1, 1, (3, n))
    src[:, : n // 3] = (0.3 + 0.15 * rng.standard_normal((3, n // 3))).clip(-0.99, 0.99)
    lo, hi = np.array([0.26, 0.26, 0.26]), np.array([0.49, 0.37, 0.37])
    trg = lo[:, None] + (hi - lo)[:, None] * rng.uniform(0, 1, (3, m))
    inside = np.flatnonzero(np.all((src >= lo[:, None]) & (src <= hi[:, None]), axis=0))
    trg[:, : min(20, len(inside))] = src[:, inside[:20]]
    return src, rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), trg


# measured at depth 3 / 4: single layer 4.0e-4 / 1.1e-3 (order 4) and 1.3e-5 /
# 3.5e-5 (order 6); double layer 1.1e-4 / 6.9e-4 (order 4) and below 1.3e-4
# (order 6).  Planted mistakes in the deep passes, on this data, at order 6
# (depth 3 / 4): the M2M child surface at the parent's radius 6.4e-4 /
# 5.9e-2, M2M without the children's point sources 2.8e-3 / 5.2e-3, M2M not
# summing the children's flux 1.3e-2 / 1.8e-2, M2L without the point sources
# 2.0e-2 / 7.3e-2; at order 4, no L2L 1.1e-2 .. 0.28 and L2L from the wrong
# parent surface 9.6e-3 .. 1.65.  None reaches the order-6 bar or a tenfold
# drop from order 4.
DEEP_ERR = {4: 6e-3, 6: 3e-4}


@pytest.mark.parametrize("D", [3, 4])
def test_deep_tree_single_layer(D):
    src, f, w, trg = _deep_cloud(111)
    ref = O.sl(src, f, w, trg, mu=0.8)
    e4 = rel(F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, D, 4, mu=0.8), ref)
    e6 = rel(F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, D, 6, mu=0.8), ref)
    assert e4 < DEEP_ERR[4] and e6 < DEEP_ERR[6] and e6 < e4 / 10, (e4, e6)


@pytest.mark.parametrize("D", [3, 4])
def test_deep_tree_double_layer_with_flux(D):
    src, _, w, trg = _deep_cloud(111)
    rng = np.random.default_rng(112)
    nrm = rng.standard_normal(src.shape)
    nrm /= np.linalg.norm(nrm, axis=0)
    phi = nrm * rng.uniform(0.5, 1.5, src.shape[1])      # n . q > 0 at every source
    assert (w * (nrm * phi).sum(axis=0)).min() > 0
    ref = O.dl(src, phi, w, nrm, trg)
    e4 = rel(F.fmm_dl(src, phi, w, nrm, trg, np.zeros(3), 1.0001, D, 4), ref)
    e6 = rel(F.fmm_dl(src, phi, w, nrm, trg, np.zeros(3), 1.0001, D, 6), ref)
    assert e4 < DEEP_ERR[4] and e6 < DEEP_ERR[6] and e6 < e4 / 10, (e4, e6)


def _two_clusters(seed, n=400, m=60):
    """Sources in two clusters (one level-2 box, and eight around the opposite
    corner); targets half in the clusters, half anywhere in the cube."""
    rng = np.random.default_rng(seed)
    src = np.concatenate([rng.uniform(-0.95, -0.55, (3, n // 2)), rng.uniform(0.3, 0.9, (3, n // 2))], axis=1)
    trg = np.concatenate([rng.uniform(-0.95, -0.55, (3, m // 2)), rng.uniform(0.3, 0.9, (3, m // 2))], axis=1)
    trg[:, ::2] = rng.uniform(-1, 1, (3, m // 2))
    return src, rng.standard_normal((3, n)), rng.uniform(0.5, 1.0, n), trg


def test_high_order_reaches_the_mixed_bar():
    """At order 10 the FMM is within 1e-7 of the direct sum (measured 1.2e-8 at
    depth 2): the pseudo-inverse cutoff (1e-10 of the largest singular value)
    keeps the rounding noise of the near-singular check-to-equivalent solves
    out of the equivalent densities (a 1e-12 cutoff leaves 4.8e-7 here)."""
    src, f, w, trg = _two_clusters(3)
    e = rel(F.fmm_sl(src, f, w, trg, np.zeros(3), 1.0001, 2, 10), O.sl(src, f, w, trg))
    assert e < 1e-7, e
