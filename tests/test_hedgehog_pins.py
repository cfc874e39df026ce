"""Pins of the singular / near-singular quadrature oracle (Sec. 3.1) against
facts fixed by the mathematics, independent of the oracle's own code.

  * interpolation reproduces polynomials of degree q-1 (values, derivatives)
                                              -> the upsampling operator U
  * the fine rule integrates degree 2q-1 exactly on every sub-interval
                                              -> fine nodes and weights
  * fine geometry of a patched sphere: radius, outward normals, total area
                                              -> fine normals and weights
  * extrapolation weights: binomial closed form for R = r and a target on the
    surface; exact for polynomials of degree p  -> e_i
  * check points on a sphere lie on the concentric spheres of radius a - s_i
                                              -> sign and scale of c_i
  * Gauss identity (constant density gives -phi inside, so its interior limit
    on the surface is -phi and the principal value -phi/2), rigid motions
    (-(U + omega x x)) on an ellipsoid and the normal density on a sphere (0
    inside), on and near the surface        -> the whole chain
"""
import math

import numpy as np
import pytest

from oracle import hedgehog as H
from paper_1909_11085_amd import workloads as W

P, RF, ETA = 8, 0.15, 2


def test_interpolation_reproduces_polynomials():
    rng = np.random.default_rng(21)
    for q in (4, 11, 16):
        t, _ = np.polynomial.legendre.leggauss(q)
        c = rng.standard_normal(q)                         # degree q-1
        x = np.concatenate([rng.uniform(-1, 1, 50), [-1.0, 1.0], t])
        poly = np.polynomial.Polynomial(c)
        B = H.lagrange_basis(t, x)
        D = H.lagrange_basis_deriv(t, x)
        assert np.abs(B @ poly(t) - poly(x)).max() < 1e-12 * np.abs(c).sum()
        assert np.abs(D @ poly(t) - poly.deriv()(x)).max() < 1e-10 * np.abs(c).sum() * q * q
        # the basis is the identity at the nodes, exactly
        assert np.array_equal(H.lagrange_basis(t, t), np.eye(q))


def test_fine_rule_integrates_polynomials():
    q = 7
    t, w = np.polynomial.legendre.leggauss(q)
    for eta in (0, 1, 2):
        s, ws = H.fine_rule(t, w, eta)
        assert len(s) == 2 ** eta * q and np.all(np.diff(s) > 0) and s.min() > -1 and s.max() < 1
        for k in range(2 * q):
            exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
            assert abs((ws * s ** k).sum() - exact) < 1e-14


def test_upsampled_sphere_geometry():
    a = 1.7
    s = W.cube_sphere(a, m=2, q=16, centre=(0.3, -0.2, 0.1))
    t, w = s.meta["nodes_1d"], s.meta["weights_1d"]
    rng = np.random.default_rng(22)
    # density: a polynomial of degree 15 in each patch variable -> upsampled exactly
    q, npatch = 16, s.meta["n_patches"]
    cu, cv = rng.standard_normal(q), rng.standard_normal(q)
    pu, pv = np.polynomial.Polynomial(cu), np.polynomial.Polynomial(cv)
    k = np.arange(s.n)
    phi = np.stack([pu(t[(k // q) % q]) * pv(t[k % q])] * 3) * np.array([[1.0], [2.0], [-1.0]])
    for eta in (1, 2):
        fx, fphi, fw, fn, L = H.upsample(s.pos, phi, t, w, eta)
        nf = (2 ** eta * q) ** 2
        assert fx.shape == (3, npatch * nf)
        r = fx - np.array([[0.3], [-0.2], [0.1]])
        rad = np.linalg.norm(r, axis=0)
        assert np.abs(rad - a).max() < 1e-11
        assert np.abs(fn - r / rad).max() < 1e-10                     # outward unit normals
        assert abs(fw.sum() - 4 * math.pi * a * a) < 1e-11 * a * a
        assert abs((L ** 2).sum() - 4 * math.pi * a * a) < 1e-11 * a * a
        sf, _ = H.fine_rule(t, w, eta)
        kk = np.arange(nf)
        want = pu(sf[kk // len(sf)]) * pv(sf[kk % len(sf)])
        got = fphi.reshape(3, npatch, nf)
        assert np.abs(got[0] - want[None, :]).max() < 1e-11 * np.abs(want).max()
        assert np.abs(got[2] + want[None, :]).max() < 1e-11 * np.abs(want).max()


def test_extrapolation_weights():
    # R = r, target on the surface: e_i = (-1)^i C(p+1, i+1)
    for p in (1, 4, 8, 12):
        nodes = 0.3 * (1 + np.arange(p + 1))
        e = H.extrapolation_weights(nodes, 0.0)
        want = np.array([(-1) ** i * math.comb(p + 1, i + 1) for i in range(p + 1)], dtype=float)
        assert np.abs(e - want).max() < 1e-10 * np.abs(want).max()
    # exact for degree <= p at any distance, R != r
    nodes = 0.12 + 0.05 * np.arange(P + 1)
    for d in (0.0, 0.04, 0.2, 0.37):
        e = H.extrapolation_weights(nodes, d)
        for k in range(P + 1):
            assert abs((e * nodes ** k).sum() - d ** k) < 1e-9 * max(1.0, d ** k)


def test_check_points_on_sphere():
    a = 2.0
    s = W.cube_sphere(a, m=2, q=16)
    t = s.meta["nodes_1d"]
    pt, u, v, d = H.on_surface_targets(s.meta["n_patches"], t)
    y, n = H.surface_point(s.pos, t, pt, u, v)
    assert np.array_equal(y, s.pos)                                    # nodes are reproduced exactly
    L = np.full(len(pt), 0.9)
    c = H.check_points(y, n, L, 5, 0.1, 0.2)
    rad = np.linalg.norm(c, axis=0)                                    # (M, 6)
    want = a - (0.1 + 0.2 * np.arange(6)) * 0.9
    assert np.abs(rad - want[None, :]).max() < 1e-10
    assert np.abs((c / rad[None] - (y / a)[:, :, None])).max() < 1e-10  # on the radial line


def _targets(surf, rng, n_on, n_near, dmax):
    """n_on node targets on the surface and n_near random near-surface targets
    up to dmax * L inside."""
    t = surf.meta["nodes_1d"]
    q = surf.meta["q"]
    pt, u, v, d = H.on_surface_targets(surf.meta["n_patches"], t)
    pick = np.sort(rng.choice(len(pt), n_on, replace=False))
    L = np.sqrt(surf.weight.reshape(-1, q * q).sum(1))
    patch = rng.integers(0, surf.meta["n_patches"], n_near).astype(np.int32)
    return (np.concatenate([pt[pick], patch]), np.concatenate([u[pick], rng.uniform(-1, 1, n_near)]),
            np.concatenate([v[pick], rng.uniform(-1, 1, n_near)]),
            np.concatenate([d[pick], rng.uniform(0, dmax, n_near) * L[patch]]))


def test_constant_density_interior_limit():
    s = W.cube_sphere(1.2, m=2, q=16)
    t, w = s.meta["nodes_1d"], s.meta["weights_1d"]
    phi0 = np.array([0.7, -0.3, 1.1])
    phi = np.repeat(phi0[:, None], s.n, axis=1)
    tg = _targets(s, np.random.default_rng(23), 150, 50, 0.3)
    out = H.singular_dl(s.pos, phi, t, w, ETA, P, RF, RF, *tg)
    assert np.abs(out + phi0[:, None]).max() < 1e-10
    # on the surface the principal value is the interior limit plus phi/2
    pv = out[:, :150] + 0.5 * phi0[:, None]
    assert np.abs(pv + 0.5 * phi0[:, None]).max() < 1e-10


def test_rigid_motion_interior_limit():
    e = W.cube_sphere(1.0, m=2, q=16, axes=(1.0, 0.8, 0.6), centre=(0.1, 0.0, -0.2))
    t, w = e.meta["nodes_1d"], e.meta["weights_1d"]
    U, om = np.array([0.2, -0.7, 0.4]), np.array([1.1, 0.3, -0.6])
    phi = U[:, None] + np.cross(om[:, None], e.pos, axis=0)
    tg = _targets(e, np.random.default_rng(24), 150, 60, 0.3)
    out, parts = H.singular_dl(e.pos, phi, t, w, ETA, P, RF, RF, *tg, return_parts=True)
    x = parts["x"]
    assert np.abs(x[:, :150] - e.pos[:, np.sort(np.random.default_rng(24).choice(e.n, 150, replace=False))]).max() == 0
    expect = -(U[:, None] + np.cross(om[:, None], x, axis=0))
    assert np.abs(out - expect).max() < 1e-9 * np.abs(expect).max()


def test_normal_density_on_sphere():
    s = W.cube_sphere(0.8, m=2, q=16)
    t, w = s.meta["nodes_1d"], s.meta["weights_1d"]
    tg = _targets(s, np.random.default_rng(25), 150, 50, 0.3)
    out = H.singular_dl(s.pos, s.normal, t, w, ETA, P, RF, RF, *tg)
    assert np.abs(out).max() < 1e-10


def test_smooth_rule_alone_fails_on_the_surface():
    """Without the check points the self-excluded smooth sum at a node is far
    from the interior limit: the quadrature is what makes the pins pass."""
    from oracle import oracle as O
    s = W.cube_sphere(1.0, m=2, q=16)
    phi0 = np.array([1.0, 0.0, 0.0])
    phi = np.repeat(phi0[:, None], s.n, axis=1)
    x = s.pos[:, ::97]
    u = O.dl(s.pos, phi, s.weight, s.normal, np.ascontiguousarray(x))
    assert np.abs(u + phi0[:, None]).max() > 1e-2
