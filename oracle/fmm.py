"""CPU oracle of the kernel-independent fast multipole method for the
single- and double-layer sums -- test infrastructure only (imported by ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark; never by the product package).

Sec. 3.1, "Far evaluation": the smooth quadrature is an N-body sum, evaluated
for all targets at once by a kernel-independent FMM.  The paper uses PVFMM and
does not describe its algorithm; this follows the published kernel-independent
method of Ying, Biros and Zorin (J. Comput. Phys. 196, 2004) on a uniform
octree:

  tree     the cube (centre c, half-width R) split into 8^D leaves; a box at
           level l has half-width h_l = R / 2^l.
  surfaces the points of a cube surface with p points per edge (6(p-1)^2 + 2
           points), scaled by alpha * h_l about the box centre:
           upward equivalent alpha = 1.05, upward check 2.95, downward
           equivalent 2.95, downward check 1.05.
  P2M      velocity of the leaf's sources at its upward check points, then
           the upward equivalent density = pinv(K_uc,ue) times it.
  M2M      velocity of the children's equivalent densities at the parent's
           upward check points, then the same pseudo-inverse at that level.
  M2L      for box B (levels 2..D), the velocity at B's downward check points
           of the upward equivalent densities of B's interaction list (children
           of the parent's neighbours that are not B's neighbours).
  L2L      plus the velocity of the parent's downward equivalent density there,
           then the downward equivalent density = pinv(K_dc,de) times it.
  L2P/P2P  each target adds the velocity of its leaf's downward equivalent
           density and the direct sum over the sources of the 27 leaves
           around its own (zero-distance pairs skipped).
Double-layer sources (the check points of the boundary solve are evaluated
this way in the paper) use the double-layer kernel in P2M and P2P.  Their
field has a net flux, sum of n . q over the sources (the flux of one stresslet
through a sphere around it is n . q), which no single-layer density carries:
each box therefore also carries a point source of that flux at its centre
(velocity sigma r / (4 pi rho^3)); its upward equivalent density represents
the flux-free rest, M2M adds the children's point sources into the parent's,
and M2L adds the point-source velocity of each interaction-list box.  For
single-layer sources every sigma is 0.

Readings: the surface radii and the pseudo-inverse are not in the paper; the
radii are the customary ones of the method, and pinv drops singular values
below 1e-10 of the largest (the single layer on a closed surface annihilates
the normal density, so the matrix is singular; from order 8 on its smallest
singular values fall below 1e-12 of the largest, where float64 determines
their singular vectors only to about 1e-4, and a lower cutoff lets that noise
into the equivalent densities: at order 10 a 1e-12 cutoff gives an error of
about 5e-7 to 3e-6 against the direct sum, 1e-10 about 1e-8 to 1e-7).  The
pseudo-inverses are formed once for a unit box and scaled by h_l (the kernel
is homogeneous of degree -1).
"""
from __future__ import annotations

import itertools

import numpy as np

ALPHA_UE, ALPHA_UC, ALPHA_DE, ALPHA_DC = 1.05, 2.95, 2.95, 1.05
PINV_RCOND = 1e-10


def surface(p):
    """(n_s, 3) points of the surface of [-1, 1]^3 with p points per edge, in
    lexicographic (i, j, k) order of the p^3 grid."""
    g = np.linspace(-1.0, 1.0, p)
    pts = [(g[i], g[j], g[k]) for i in range(p) for j in range(p) for k in range(p)
           if min(i, j, k) == 0 or max(i, j, k) == p - 1]
    return np.array(pts)


def kernel_matrix(x, y, mu=1.0):
    """(3 n_x, 3 n_y) matrix of the single-layer kernel (eq. sl_stokes) from
    points y to points x, index 3*point + component; zero at zero distance."""
    r = x[:, None, :] - y[None, :, :]
    rho2 = (r ** 2).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        ri = np.where(rho2 > 0, 1.0 / np.sqrt(rho2), 0.0)
    K = (np.eye(3)[None, None, :, :] * ri[:, :, None, None]
         + r[:, :, :, None] * r[:, :, None, :] * (ri ** 3)[:, :, None, None]) / (8.0 * np.pi * mu)
    return K.transpose(0, 2, 1, 3).reshape(3 * len(x), 3 * len(y))


def operators(p, mu=1.0):
    """Pseudo-inverses for a box of half-width 1 (check -> equivalent), upward
    and downward."""
    s = surface(p)
    up = np.linalg.pinv(kernel_matrix(ALPHA_UC * s, ALPHA_UE * s, mu), rcond=PINV_RCOND)
    down = np.linalg.pinv(kernel_matrix(ALPHA_DC * s, ALPHA_DE * s, mu), rcond=PINV_RCOND)
    return s, up, down


def dl_matrix(x, y, nrm):
    """(3 n_x, 3 n_y) matrix of the double-layer kernel (after eq.
    double_layer_int_eq) from points y with normals nrm (n_y, 3) to points x:
    6/(8 pi) r (r.n) r^T / rho^5; zero at zero distance."""
    r = x[:, None, :] - y[None, :, :]
    rho2 = (r ** 2).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        ri5 = np.where(rho2 > 0, rho2 ** -2.5, 0.0)
    rn = (r * nrm[None, :, :]).sum(-1)
    K = 6.0 / (8.0 * np.pi) * (rn * ri5)[:, :, None, None] * r[:, :, :, None] * r[:, :, None, :]
    return K.transpose(0, 2, 1, 3).reshape(3 * len(x), 3 * len(y))


def source_velocity(x, y, sigma):
    """Velocity (3 n_x flattened, index 3*point + component) at points x of a
    point source of flux sigma at y: sigma r / (4 pi rho^3)."""
    r = x - np.asarray(y, dtype=np.float64)[None, :]
    rho = np.linalg.norm(r, axis=1)
    return (sigma * r / (4.0 * np.pi * rho[:, None] ** 3)).reshape(-1)


def _leaf_index(x, c, R, D):
    n = 2 ** D
    idx = np.floor((x - (np.asarray(c) - R)[:, None]) / (2.0 * R / n)).astype(np.int64)
    return np.clip(idx, 0, n - 1)


def fmm_sl(src, f, w, trg, c, R, D, p, mu=1.0):
    """Single-layer velocity (3, n_trg) at the targets from the sources (q =
    w f), by the kernel-independent FMM on the uniform tree of depth D >= 2
    over the cube (c, R) that holds every point."""
    return _fmm(src, f, w, None, trg, c, R, D, p, mu)


def fmm_dl(src, phi, w, nrm, trg, c, R, D, p):
    """Double-layer velocity (3, n_trg) from the sources (q = w phi, normals
    nrm (3, n_src)) by the same FMM."""
    return _fmm(src, phi, w, nrm, trg, c, R, D, p, 1.0)


def _fmm(src, f, w, nrm, trg, c, R, D, p, mu):
    src, trg = np.asarray(src, dtype=np.float64), np.asarray(trg, dtype=np.float64)
    q = (np.asarray(w)[None, :] * np.asarray(f)).T                 # (n_src, 3)
    c = np.asarray(c, dtype=np.float64)
    if nrm is None:
        src_matrix = lambda x, ms: kernel_matrix(x, src[:, ms].T, mu)
    else:
        nrm = np.asarray(nrm, dtype=np.float64)
        src_matrix = lambda x, ms: dl_matrix(x, src[:, ms].T, nrm[:, ms].T)
    s, up, down = operators(p, mu)
    ns = len(s)
    n_leaf = 2 ** D
    si, ti = _leaf_index(src, c, R, D), _leaf_index(trg, c, R, D)
    leaf_src = {}
    for m in range(src.shape[1]):
        leaf_src.setdefault(tuple(si[:, m]), []).append(m)

    def centre(l, idx):
        h = R / 2 ** l
        return c - R + (2 * np.asarray(idx) + 1) * h

    # upward pass: equivalent densities (ns, 3) and point-source fluxes per
    # non-empty box, per level
    ue = [dict() for _ in range(D + 1)]
    sig = [dict() for _ in range(D + 1)]
    for idx, ms in leaf_src.items():
        h = R / 2 ** D
        ctr = centre(D, idx)
        chk = ctr + ALPHA_UC * h * s
        sigma = 0.0 if nrm is None else float((nrm[:, ms].T * q[ms]).sum())
        v = src_matrix(chk, ms) @ q[ms].reshape(-1) - source_velocity(chk, ctr, sigma)
        ue[D][idx] = (h * up @ v).reshape(ns, 3)
        sig[D][idx] = sigma
    for l in range(D - 1, 1, -1):
        h = R / 2 ** l
        parents = {tuple(np.asarray(ci) // 2) for ci in ue[l + 1]}
        for pidx in parents:
            ctr = centre(l, pidx)
            chk = ctr + ALPHA_UC * h * s
            v = np.zeros(3 * ns)
            sigma = 0.0
            for off in itertools.product((0, 1), repeat=3):
                ci = tuple(2 * np.asarray(pidx) + off)
                if ci in ue[l + 1]:
                    cc = centre(l + 1, ci)
                    v += kernel_matrix(chk, cc + ALPHA_UE * (h / 2) * s, mu) @ ue[l + 1][ci].reshape(-1)
                    v += source_velocity(chk, cc, sig[l + 1][ci])
                    sigma += sig[l + 1][ci]
            v -= source_velocity(chk, ctr, sigma)
            ue[l][pidx] = (h * up @ v).reshape(ns, 3)
            sig[l][pidx] = sigma

    # downward pass: equivalent densities of every box that holds targets
    need = [set() for _ in range(D + 1)]
    for m in range(trg.shape[1]):
        idx = ti[:, m]
        for l in range(D, 1, -1):
            need[l].add(tuple(idx >> (D - l)))
    de = [dict() for _ in range(D + 1)]
    for l in range(2, D + 1):
        h = R / 2 ** l
        nb = 2 ** l
        for idx in need[l]:
            ctr = centre(l, idx)
            chk = ctr + ALPHA_DC * h * s
            v = np.zeros(3 * ns)
            pidx = tuple(np.asarray(idx) // 2)
            for poff in itertools.product((-1, 0, 1), repeat=3):
                pn = np.asarray(pidx) + poff
                if np.any(pn < 0) or np.any(pn >= nb // 2):
                    continue
                for coff in itertools.product((0, 1), repeat=3):
                    a = tuple(2 * pn + coff)
                    if max(abs(a[k] - idx[k]) for k in range(3)) <= 1 or a not in ue[l]:
                        continue
                    v += kernel_matrix(chk, centre(l, a) + ALPHA_UE * h * s, mu) @ ue[l][a].reshape(-1)
                    v += source_velocity(chk, centre(l, a), sig[l][a])
            if l > 2:
                v += kernel_matrix(chk, centre(l - 1, pidx) + ALPHA_DE * (2 * h) * s, mu) @ de[l - 1][pidx].reshape(-1)
            de[l][idx] = (h * down @ v).reshape(ns, 3)

    # evaluation: L2P and P2P
    out = np.zeros((3, trg.shape[1]))
    h = R / 2 ** D
    for m in range(trg.shape[1]):
        idx = tuple(ti[:, m])
        x = trg[:, m]
        u = kernel_matrix(x[None, :], centre(D, idx) + ALPHA_DE * h * s, mu) @ de[D][idx].reshape(-1)
        near = []
        for off in itertools.product((-1, 0, 1), repeat=3):
            nbr = tuple(np.asarray(idx) + off)
            if nbr in leaf_src:
                near.extend(leaf_src[nbr])
        if near:
            u = u + src_matrix(x[None, :], near) @ q[near].reshape(-1)
        out[:, m] = u
    return out
