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
"""
import numpy as np

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
