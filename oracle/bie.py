"""FP64 CPU oracle of the discretised boundary integral equation and its GMRES
solve -- test infrastructure only (imported by ``tests/``, the smoke check and
the CPU-baseline leg of the benchmark; never by the product package).

Sec. 2.1.2, eq. (double_layer_int_eq), and Sec. 3.1, "Discretizing the integral
equation", eq. (int_eq_disc): the velocity inside a closed surface is the
double layer u = D phi of a density phi found from its boundary values g.  The
discrete operator at the patch nodes y_l is the check-point quadrature (the
limit from inside, ``oracle.hedgehog.singular_dl``) plus a rank-completing term,
and GMRES solves the system matrix-free.

Readings (the paper's signs are not consistent with its kernel):
  * With this kernel the limit from inside is (D_pv - I/2) phi (constant phi
    gives -phi).  The interior Dirichlet problem is therefore
        (L_in - N) phi = g,   L_in phi = limit from inside of D phi,
        (N phi)(x) = n(x) * integral over the surface of n(y) . phi(y),
    the paper's (I/2 + D + N) phi = g with D of the opposite sign.  The range
    of L_in is orthogonal to n, so compatible data (integral of g . n = 0)
    give N phi = 0 at the solution whatever the sign of N; the minus sign puts
    the one eigenvalue N moves (-|surface|) on the same side as the rest of
    the spectrum (-1 .. 0).
  * The integral in N uses the patch rule at the nodes, with the normals and
    weights of the patch polynomial (the fine discretisation with eta = 0).
  * GMRES starts from phi = 0, without restarts, and stops when the residual
    estimate |g - A phi| / |g| drops to rtol or after max_iter iterations (the
    paper caps the solve at 30).
"""
from __future__ import annotations

import numpy as np

from oracle import hedgehog as H


def node_geometry(node_xyz, t, w):
    """Unit normals (3, N) and weights (N) at the patch nodes, from the patch
    polynomial (the eta = 0 fine discretisation is the nodes themselves)."""
    _, _, nw, nn, _ = H.upsample(node_xyz, np.zeros_like(node_xyz), t, w, 0)
    return nn, nw


def apply_interior(node_xyz, phi, t, w, eta, p, R_frac, r_frac):
    """L_in phi at every node: the check-point quadrature on the surface."""
    return H.singular_dl(node_xyz, phi, t, w, eta, p, R_frac, r_frac)


def apply_n(phi, nn, nw):
    """(N phi)(y_l) = n_l sum_m w_m n_m . phi_m."""
    return nn * float((nw * (nn * phi).sum(0)).sum())


def operator_matrix(node_xyz, t, w, eta, p, R_frac, r_frac):
    """The dense matrix of (L_in - N), column by column from unit densities
    (flattened component-major: index c*N + l)."""
    n = node_xyz.shape[1]
    nn, nw = node_geometry(node_xyz, t, w)
    A = np.empty((3 * n, 3 * n))
    for c in range(3):
        for m in range(n):
            e = np.zeros((3, n))
            e[c, m] = 1.0
            A[:, c * n + m] = (apply_interior(node_xyz, e, t, w, eta, p, R_frac, r_frac)
                               - apply_n(e, nn, nw)).reshape(-1)
    return A


def gmres(matvec, g, max_iter, rtol):
    """Textbook GMRES (Saad): Arnoldi with modified Gram-Schmidt, Givens
    rotations on the Hessenberg matrix, x0 = 0.  Returns (x, residual
    estimates |r_k| / |g| for k = 0..iterations)."""
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    beta = np.linalg.norm(g)
    hist = [1.0]
    if beta == 0.0:
        return np.zeros_like(g), hist
    V = [g / beta]
    Hm = np.zeros((max_iter + 1, max_iter))
    cs, sn = np.zeros(max_iter), np.zeros(max_iter)
    s = np.zeros(max_iter + 1)
    s[0] = beta
    k = 0
    for j in range(max_iter):
        wv = matvec(V[j])
        for i in range(j + 1):
            Hm[i, j] = wv @ V[i]
            wv = wv - Hm[i, j] * V[i]
        hnext = np.linalg.norm(wv)
        Hm[j + 1, j] = hnext
        for i in range(j):                              # earlier rotations on the new column
            a, b = Hm[i, j], Hm[i + 1, j]
            Hm[i, j], Hm[i + 1, j] = cs[i] * a + sn[i] * b, -sn[i] * a + cs[i] * b
        den = np.hypot(Hm[j, j], Hm[j + 1, j])
        cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
        Hm[j, j], Hm[j + 1, j] = den, 0.0
        s[j + 1] = -sn[j] * s[j]
        s[j] = cs[j] * s[j]
        k = j + 1
        hist.append(abs(s[j + 1]) / beta)
        if hist[-1] <= rtol or hnext == 0.0:         # converged, or the Krylov space is invariant
            break
        V.append(wv / hnext)
    y = np.linalg.solve(np.triu(Hm[:k, :k]), s[:k])
    x = sum(y[i] * V[i] for i in range(k))
    return x, hist


def stokeslet(x, x0, F, mu=1.0):
    """Velocity of a point force F at x0 (the single-layer kernel of eq.
    sl_stokes): (F/rho + r (r.F)/rho^3) / (8 pi mu), r = x - x0."""
    r = x - np.asarray(x0, dtype=np.float64)[:, None]
    rho = np.linalg.norm(r, axis=0)
    F = np.asarray(F, dtype=np.float64)[:, None]
    return (F / rho + r * (r * F).sum(0) / rho ** 3) / (8.0 * np.pi * mu)
