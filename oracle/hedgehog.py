"""FP64 CPU oracle of the singular / near-singular double-layer quadrature --
test infrastructure only (imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package).

Sec. 3.1, "Singular and near-singular integral quadrature": to evaluate the
double-layer velocity at a point x on or near the surface,
  1. upsample the density with the patch's q-th order interpolant onto k = 4^eta
     sub-squares of every patch, each carrying the patch's own tensor-product
     rule (the fine discretisation, phi_up = U phi);
  2. take the closest surface point y = P(u*, v*) (y = x on the surface);
  3. place p + 1 check points c_i = y - (R + i r) n(u*, v*), i = 0..p, on the
     inward side of the outward normal n;
  4. evaluate the smooth quadrature of eq. (smooth_double_layer_int_eq_patches_disc)
     over the fine discretisation at every check point (eq. quad_check_points);
  5. extrapolate to x with 1-D polynomial weights e_i (eq. sing-quad).
R and r are fractions of the patch size L, the square root of the area of the
patch holding y (Sec. 5.1 parameters).

Readings (the paper is silent on them):
  * A patch is the tensor-product polynomial of degree q-1 in each variable
    through its q x q nodes; its fine nodes, normals X_u x X_v / |X_u x X_v|
    and weights w_i w_j / 4^eta * |X_u x X_v| all come from that polynomial.
  * The closest point is an input: a target is (patch, u*, v*, d) and sits at
    x = y - d n, d >= 0 its distance inside.  On-surface targets at the patch
    nodes are (patch, t_i, t_j, 0).
  * The extrapolation variable is the distance along -n: check point i sits at
    s_i = (R + i r) L, the target at s = d; e_i is the Lagrange basis polynomial
    of the nodes s_0..s_p evaluated at d.
  * The value returned is the limit from the side the check points lie on (the
    interior of a closed surface with outward normals), so a constant density
    gives -phi there, and the principal value on the surface is that limit
    plus phi / 2.

Every step is a plain loop or a library primitive (einsum, the C double-layer
sum of ``oracle.dl``); nothing is blocked, fused or reordered.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


# ------------------------------------------------------------- step 1: U
def lagrange_basis(t, x):
    """B[a, m] = l_m(x_a), the Lagrange basis polynomials of the nodes t
    evaluated at the points x (product form)."""
    t = np.asarray(t, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    q = len(t)
    B = np.ones((len(x), q))
    for m in range(q):
        for k in range(q):
            if k != m:
                B[:, m] *= (x - t[k]) / (t[m] - t[k])
    return B


def lagrange_basis_deriv(t, x):
    """D[a, m] = l_m'(x_a): derivative of the product form by the product rule,
    sum over j != m of 1/(t_m - t_j) times the product over k != m, j."""
    t = np.asarray(t, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    q = len(t)
    D = np.zeros((len(x), q))
    for m in range(q):
        for j in range(q):
            if j == m:
                continue
            term = np.full(len(x), 1.0 / (t[m] - t[j]))
            for k in range(q):
                if k != m and k != j:
                    term *= (x - t[k]) / (t[m] - t[k])
            D[:, m] += term
    return D


def fine_rule(t, w, eta):
    """The patch rule (t, w) on [-1, 1] repeated on each of the 2^eta equal
    sub-intervals: nodes -1 + (2a + 1 + t_j) / 2^eta, weights w_j / 2^eta,
    ordered sub-interval major."""
    ns = 2 ** eta
    t = np.asarray(t, dtype=np.float64)
    s = np.concatenate([-1.0 + (2 * a + 1 + t) / ns for a in range(ns)])
    ws = np.concatenate([np.asarray(w, dtype=np.float64) / ns for _ in range(ns)])
    return s, ws


def _patches(a, n_patches, q):
    """(3, n_patches*q*q) patch-major -> (3, n_patches, q, q)."""
    return np.asarray(a, dtype=np.float64).reshape(3, n_patches, q, q)


def upsample(node_xyz, density, t, w, eta):
    """Fine discretisation of every patch (step 1).

    node_xyz, density: (3, n_patches*q*q), patch-major, node k = i*q + j at
    (u, v) = (t_i, t_j).  Returns fine positions, densities U phi, weights and
    unit normals, each patch-major with (2^eta q)^2 fine nodes per patch (node
    I*(2^eta q) + J at (s_I, s_J) of ``fine_rule``), and the patch sizes L."""
    q = len(t)
    n_patches = np.asarray(node_xyz).shape[1] // (q * q)
    s, ws = fine_rule(t, w, eta)
    B = lagrange_basis(t, s)
    D = lagrange_basis_deriv(t, s)
    X = _patches(node_xyz, n_patches, q)
    F = _patches(density, n_patches, q)
    Xf = np.einsum("Im,Jl,cpml->cpIJ", B, B, X)
    Xu = np.einsum("Im,Jl,cpml->cpIJ", D, B, X)
    Xv = np.einsum("Im,Jl,cpml->cpIJ", B, D, X)
    Ff = np.einsum("Im,Jl,cpml->cpIJ", B, B, F)
    c = np.cross(Xu, Xv, axis=0)
    area_el = np.linalg.norm(c, axis=0)
    nrm = c / area_el
    wf = np.outer(ws, ws)[None, :, :] * area_el
    L = np.sqrt(wf.sum(axis=(1, 2)))
    nf = n_patches * len(s) ** 2
    return (Xf.reshape(3, nf), Ff.reshape(3, nf), wf.reshape(nf), nrm.reshape(3, nf), L)


# ---------------------------------------------------- steps 2 and 3: c_i
def surface_point(node_xyz, t, patch, u, v):
    """y = P(u, v) and the unit normal X_u x X_v / |X_u x X_v| for each target
    (patch[a], u[a], v[a])."""
    q = len(t)
    n_patches = np.asarray(node_xyz).shape[1] // (q * q)
    X = _patches(node_xyz, n_patches, q)[:, np.asarray(patch)]       # (3, M, q, q)
    Bu, Bv = lagrange_basis(t, u), lagrange_basis(t, v)
    Du, Dv = lagrange_basis_deriv(t, u), lagrange_basis_deriv(t, v)
    y = np.einsum("am,al,caml->ca", Bu, Bv, X)
    xu = np.einsum("am,al,caml->ca", Du, Bv, X)
    xv = np.einsum("am,al,caml->ca", Bu, Dv, X)
    c = np.cross(xu, xv, axis=0)
    return y, c / np.linalg.norm(c, axis=0)


def check_points(y, n, L, p, R_frac, r_frac):
    """c[:, a, i] = y_a - (R + i r) n_a with R = R_frac L_a, r = r_frac L_a,
    i = 0..p (step 3)."""
    L = np.asarray(L, dtype=np.float64)
    s = (R_frac + r_frac * np.arange(p + 1))[None, :] * L[:, None]           # (M, p+1)
    return y[:, :, None] - s[None, :, :] * n[:, :, None]


# ---------------------------------------------------------- step 5: e_i
def extrapolation_weights(nodes, x):
    """e_i = l_i(x) for the 1-D nodes (the distances of the check points along
    -n) and the target distance x (eq. sing-quad)."""
    return lagrange_basis(nodes, [x])[0]


# ------------------------------------------------------------- together
def on_surface_targets(n_patches, t):
    """(patch, u, v, d) of every patch node, in node order."""
    q = len(t)
    k = np.arange(n_patches * q * q)
    return (k // (q * q)).astype(np.int32), np.asarray(t)[(k // q) % q], np.asarray(t)[k % q], np.zeros(len(k))


def singular_dl(node_xyz, density, t, w, eta, p, R_frac, r_frac, patch=None, u=None, v=None, d=None,
                return_parts=False):
    """Double-layer velocity at targets on or near the surface (steps 1-5).

    The targets default to every patch node on the surface.  Returns (3, M);
    with return_parts also a dict with the fine discretisation, the check
    points (3, M, p+1) and their velocities (3, M, p+1)."""
    q = len(t)
    n_patches = np.asarray(node_xyz).shape[1] // (q * q)
    if patch is None:
        patch, u, v, d = on_surface_targets(n_patches, t)
    patch = np.asarray(patch)
    d = np.asarray(d, dtype=np.float64)
    fx, fphi, fw, fn, Lp = upsample(node_xyz, density, t, w, eta)
    y, n = surface_point(node_xyz, t, patch, u, v)
    L = Lp[patch]
    c = check_points(y, n, L, p, R_frac, r_frac)
    M = len(patch)
    uc = O.dl(fx, fphi, fw, fn, np.ascontiguousarray(c.reshape(3, M * (p + 1)))).reshape(3, M, p + 1)
    out = np.empty((3, M))
    base = R_frac + r_frac * np.arange(p + 1)
    for a in range(M):
        e = extrapolation_weights(base * L[a], d[a])
        out[:, a] = uc[:, a, :] @ e
    if not return_parts:
        return out
    return out, dict(fine=(fx, fphi, fw, fn), L=Lp, y=y, n=n, check=c, check_vel=uc,
                     x=y - d[None, :] * n)
