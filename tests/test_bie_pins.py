"""Pins of the boundary-integral oracle (eq. double_layer_int_eq and eq.
int_eq_disc, GMRES) against facts fixed by linear algebra and Stokes theory,
independent of the oracle's own code.

  * GMRES's k-step iterate minimises |g - A x| over the Krylov space: equal to
    a least-squares solve over an explicit, QR-orthonormalised Krylov basis;
    its residual estimates are the true residuals; it reaches the dense solve
                                                   -> the Arnoldi/Givens code
  * the dense operator, assembled column by column, acts like the matrix-free
    one                                            -> ordering, the N term
  * rigid motions are eigenvectors of A with eigenvalue -1 (D of a rigid motion
    is minus it inside, and their normal flux is 0); on a sphere the normal
    field has eigenvalue -(surface area)           -> signs of L_in and N
  * an exterior point force gives boundary data whose solve reproduces the
    point force's velocity inside                  -> the interior Dirichlet
                                                      problem as a whole
"""
import math

import numpy as np

from oracle import bie as B
from oracle import oracle as O
from paper_1909_11085_amd import workloads as W

ETA, P, RF = 2, 8, 0.15


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_gmres_is_the_krylov_least_squares_solution():
    rng = np.random.default_rng(31)
    n = 120
    A = -0.5 * np.eye(n) + 0.25 * rng.standard_normal((n, n)) / math.sqrt(n)
    g = rng.standard_normal(n)
    for k in (1, 4, 9, 15):
        xk, hk = B.gmres(lambda v: A @ v, g, k, 0.0)
        assert len(hk) == k + 1
        K = np.empty((n, k))
        v = g.copy()
        for i in range(k):
            K[:, i] = v
            v = A @ v
        Q, _ = np.linalg.qr(K)
        y = np.linalg.lstsq(A @ Q, g, rcond=None)[0]
        xls = Q @ y
        assert rel(xk, xls) < 1e-9
        true = np.linalg.norm(g - A @ xk) / np.linalg.norm(g)
        assert abs(hk[-1] - true) <= 1e-12 + 1e-9 * true
        assert np.all(np.diff(hk) <= 1e-15)
    x, hist = B.gmres(lambda v: A @ v, g, 80, 1e-14)
    assert hist[-1] <= 1e-14 and len(hist) < 81
    assert rel(x, np.linalg.solve(A, g)) < 1e-11


def test_gmres_special_cases():
    g = np.arange(1.0, 7.0)
    x, h = B.gmres(lambda v: 2.0 * v, g, 10, 0.0)        # invariant after one step
    assert len(h) == 2 and rel(x, g / 2) < 1e-15 and h[-1] == 0.0
    x, h = B.gmres(lambda v: v, np.zeros(6), 10, 0.0)     # zero data
    assert np.all(x == 0) and h == [1.0]


def test_dense_operator_matches_matrix_free():
    s = W.cube_sphere(1.0, m=1, q=4, axes=(1.0, 0.9, 0.7))
    t, w = s.meta["nodes_1d"], s.meta["weights_1d"]
    A = B.operator_matrix(s.pos, t, w, 1, 4, 0.2, 0.1)
    phi = np.random.default_rng(32).standard_normal((3, s.n))
    nn, nw = B.node_geometry(s.pos, t, w)
    mf = B.apply_interior(s.pos, phi, t, w, 1, 4, 0.2, 0.1) - B.apply_n(phi, nn, nw)
    assert rel(A @ phi.reshape(-1), mf.reshape(-1)) < 1e-13
    # on a well-resolved surface the node geometry of the patch polynomial is the exact one
    f = W.cube_sphere(1.0, m=2, q=16, axes=(1.0, 0.9, 0.7))
    fn, fw = B.node_geometry(f.pos, f.meta["nodes_1d"], f.meta["weights_1d"])
    assert np.abs(fn - f.normal).max() < 1e-9 and rel(fw, f.weight) < 1e-10


def test_operator_eigenvectors():
    s = W.cube_sphere(1.0, m=2, q=8, axes=(1.0, 0.8, 0.6))
    t, w = s.meta["nodes_1d"], s.meta["weights_1d"]
    nn, nw = B.node_geometry(s.pos, t, w)
    U, om = np.array([0.2, -0.7, 0.4]), np.array([1.1, 0.3, -0.6])
    rig = U[:, None] + np.cross(om[:, None], s.pos, axis=0)
    A_rig = B.apply_interior(s.pos, rig, t, w, ETA, P, RF, RF) - B.apply_n(rig, nn, nw)
    assert rel(A_rig, -rig) < 1e-4                                    # q = 8: measured 1.7e-5
    assert abs(float((nw * (nn * rig).sum(0)).sum())) < 1e-12 * np.abs(rig).max()
    sph = W.cube_sphere(0.9, m=2, q=8)
    nn, nw = B.node_geometry(sph.pos, t, w)
    A_n = B.apply_interior(sph.pos, nn, t, w, ETA, P, RF, RF) - B.apply_n(nn, nn, nw)
    area = 4 * math.pi * 0.9 ** 2
    assert rel(A_n, -area * nn) < 1e-4


def test_interior_dirichlet_problem():
    """Boundary data of a point force outside the surface: the solved density's
    double layer reproduces the point force's velocity inside."""
    s = W.cube_sphere(1.0, m=2, q=8)
    t, w = s.meta["nodes_1d"], s.meta["weights_1d"]
    nn, nw = B.node_geometry(s.pos, t, w)
    x0, F = np.array([1.6, 0.7, -0.4]), np.array([0.3, -1.0, 0.5])
    g = B.stokeslet(s.pos, x0, F)
    assert abs(float((nw * (nn * g).sum(0)).sum())) < 1e-10          # compatible data

    def mv(v):
        v = v.reshape(3, -1)
        return (B.apply_interior(s.pos, v, t, w, ETA, P, RF, RF) - B.apply_n(v, nn, nw)).reshape(-1)

    phi, hist = B.gmres(mv, g.reshape(-1), 15, 1e-12)
    phi = phi.reshape(3, -1)
    assert hist[-1] < 1e-4
    rng = np.random.default_rng(33)
    xin = rng.standard_normal((3, 40))
    xin *= 0.6 * rng.uniform(0, 1, 40) ** (1 / 3) / np.linalg.norm(xin, axis=0)
    u = O.dl(s.pos, phi, s.weight, s.normal, xin)
    ue = B.stokeslet(xin, x0, F)
    assert np.abs(u - ue).max() < 1e-4 * np.abs(ue).max()
    # N phi vanishes at the solution of compatible data
    assert abs(float((nw * (nn * phi).sum(0)).sum())) < 1e-4 * np.abs(phi).max()
