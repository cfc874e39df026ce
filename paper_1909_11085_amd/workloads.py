"""Seeded synthetic inputs for the Stokes kernel sums.

This module only builds inputs: surface quadrature nodes with weights and
normals, cell placements, random densities, group ids, the octree leaf layout
and interaction lists.  It holds none of the kernel-sum arithmetic, and both
the HIP library's tests and the CPU oracle's tests draw their inputs from it.

Shapes follow the paper's workloads:
  * red blood cells sampled at 544 quadrature points each (Sec. 5.1 setup:
    spherical-harmonic order 16), here an Evans-Fung biconcave surface on a
    17 x 32 Gauss-Legendre(cos theta) x uniform(phi) grid;
  * vessel-wall tensor-product polynomial patches with a tensor-product
    quadrature rule on each patch (Sec. 3.1), here an open straight cylinder
    split into 64 x 64 patches of 16 x 16 Gauss-Legendre nodes;
  * cells at random orientation (Sec. 5.1, "filling the vessel"), here uniform
    on SO(3), placed by random sequential addition of disjoint bounding spheres;
  * the FMM near field (Sec. 3.1, "Far evaluation"): an adaptive octree with
    at most 256 points per leaf and a per-leaf interaction list.

Arrays are structure-of-arrays float64 of shape (3, N); group ids int32.
RNG: numpy PCG64 ``default_rng(seed)``; draw order placement -> rotations ->
densities -> reference velocities -> finite-difference coordinates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Evans-Fung biconcave shape constants (radius R and thickness coefficients).
EF_R = 3.91
EF_C0, EF_C2, EF_C4 = 0.207, 2.003, -1.123
RBC_ORDER = 16                       # 17 x 32 = 544 nodes per cell


# ----------------------------------------------------------------------------
# Surfaces of revolution: X(theta, phi) = (rho(theta) cos phi, rho(theta) sin phi, z(theta))
# ----------------------------------------------------------------------------
def _revolution_quadrature(order, rho_fn, drho_fn, z_fn, dz_fn):
    """Nodes, area weights and outward normals of a surface of revolution.

    cos(theta) at (order+1) Gauss-Legendre nodes, phi at 2*order uniform
    nodes.  With t = cos(theta), dtheta = -dt/sin(theta), so the area weight is
    w = w_GL * (2 pi / n_phi) * |X_theta x X_phi| / sin(theta), and
    X_theta x X_phi = rho * (-z' cos phi, -z' sin phi, rho') is outward for the
    shapes used here (rho = R sin(theta) > 0, z decreasing from the north pole).
    """
    n_t, n_p = order + 1, 2 * order
    t, wt = np.polynomial.legendre.leggauss(n_t)
    theta = np.arccos(t)[::-1]          # north pole first
    wt = wt[::-1]
    phi = 2.0 * np.pi * np.arange(n_p) / n_p
    TH, PH = np.meshgrid(theta, phi, indexing="ij")      # (n_t, n_p), theta-major
    W_T = np.repeat(wt[:, None], n_p, axis=1)
    rho, drho = rho_fn(TH), drho_fn(TH)
    z, dz = z_fn(TH), dz_fn(TH)
    sin_t = np.sin(TH)
    pts = np.stack([rho * np.cos(PH), rho * np.sin(PH), z]).reshape(3, -1)
    tang = np.sqrt(dz * dz + drho * drho)               # |X_theta x X_phi| / rho
    nrm = np.stack([-dz * np.cos(PH), -dz * np.sin(PH), drho]) / tang
    # |X_theta x X_phi| / sin(theta) = (rho / sin(theta)) * tang
    w = W_T * (2.0 * np.pi / n_p) * (rho / sin_t) * tang
    return pts, w.reshape(-1), nrm.reshape(3, -1)


def sphere_surface(radius=1.0, order=RBC_ORDER):
    """Sphere of the given radius centred at the origin: (points, weights, normals)."""
    a = float(radius)
    return _revolution_quadrature(
        order,
        lambda th: a * np.sin(th), lambda th: a * np.cos(th),
        lambda th: a * np.cos(th), lambda th: -a * np.sin(th))


def evans_fung_surface(order=RBC_ORDER, R=EF_R, c0=EF_C0, c2=EF_C2, c4=EF_C4):
    """Biconcave Evans-Fung cell centred at the origin, axis z.

    x = R sin(t) cos(p), y = R sin(t) sin(p),
    z = (R/2) cos(t) (c0 + c2 sin^2 t + c4 sin^4 t), derivatives analytic.
    """
    def P(s):
        return c0 + c2 * s + c4 * s * s

    def dP(s):
        return c2 + 2.0 * c4 * s

    def z_fn(th):
        return 0.5 * R * np.cos(th) * P(np.sin(th) ** 2)

    def dz_fn(th):
        s, c = np.sin(th), np.cos(th)
        return 0.5 * R * s * (-P(s * s) + 2.0 * c * c * dP(s * s))

    return _revolution_quadrature(
        order, lambda th: R * np.sin(th), lambda th: R * np.cos(th), z_fn, dz_fn)


def evans_fung_volume(R=EF_R, c0=EF_C0, c2=EF_C2, c4=EF_C4):
    """Closed-form enclosed volume pi R^3 (2 c0/3 + 4 c2/15 + 16 c4/105)."""
    return math.pi * R ** 3 * (2.0 * c0 / 3.0 + 4.0 * c2 / 15.0 + 16.0 * c4 / 105.0)


# ----------------------------------------------------------------------------
# Random rotations and placement
# ----------------------------------------------------------------------------
def random_rotations(rng, n):
    """n rotation matrices uniform on SO(3): unit quaternions from 4 iid N(0,1)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rsa_centres(rng, n, radius, lo, hi, inside=None, batch=4096, max_tries=20_000_000):
    """Random sequential addition of n disjoint spheres (|c_i - c_j| >= 2 radius).

    Candidates are drawn uniformly in the box [lo, hi] (3-vectors) and kept if
    ``inside(c)`` (optional vectorised predicate) holds and they clear every
    accepted centre.  A uniform grid with cell side 2*radius makes each check
    look at 27 cells.  Deterministic for a given rng state.
    """
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    d2min = (2.0 * radius) ** 2
    cell = 2.0 * radius
    dims = np.maximum(1, np.ceil((hi - lo) / cell).astype(int))
    cap = 8
    grid = -np.ones((dims[0] + 2, dims[1] + 2, dims[2] + 2, cap), dtype=np.int64)
    fill = np.zeros(grid.shape[:3], dtype=np.int64)
    cent = np.zeros((n, 3))     # rows not yet placed are read only under a mask
    k = 0
    tries = 0
    offs = np.array([[i, j, l] for i in (-1, 0, 1) for j in (-1, 0, 1) for l in (-1, 0, 1)])
    while k < n:
        if tries > max_tries:
            raise RuntimeError(f"RSA placed only {k} of {n} spheres in {tries} tries")
        c = lo + (hi - lo) * rng.random((batch, 3))
        tries += batch
        if inside is not None:
            c = c[inside(c)]
        if len(c) == 0:
            continue
        gi = np.clip(((c - lo) / cell).astype(int), 0, dims - 1) + 1        # (B, 3), padded grid
        nb = gi[:, None, :] + offs[None, :, :]                               # (B, 27, 3)
        ids = grid[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(len(c), -1)  # (B, 27*cap)
        valid = ids >= 0
        other = cent[np.where(valid, ids, 0)]                                # (B, 27*cap, 3)
        d2 = ((other - c[:, None, :]) ** 2).sum(-1)
        ok = ~np.any(valid & (d2 < d2min), axis=1)
        acc_batch = []
        for b in np.nonzero(ok)[0]:
            if k >= n:
                break
            cb = c[b]
            if acc_batch:
                prev = cent[acc_batch]
                if np.any(((prev - cb) ** 2).sum(-1) < d2min):
                    continue
            g = gi[b]
            if fill[g[0], g[1], g[2]] >= cap:
                continue
            cent[k] = cb
            grid[g[0], g[1], g[2], fill[g[0], g[1], g[2]]] = k
            fill[g[0], g[1], g[2]] += 1
            acc_batch.append(k)
            k += 1
    return cent, tries


@dataclass
class PointSet:
    """Quadrature points of a set of surfaces (sources and/or targets)."""
    pos: np.ndarray            # (3, N) float64
    weight: np.ndarray         # (N,) float64 area quadrature weights
    normal: np.ndarray         # (3, N) float64 outward unit normals
    group: np.ndarray          # (N,) int32 surface (cell or patch) id
    group_h: np.ndarray        # (n_groups,) float64 mesh spacing sqrt(area / n_points)
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.pos.shape[1]


def place_cells(rng, n_cells, container, order=RBC_ORDER):
    """n_cells Evans-Fung cells with RSA centres and uniform random rotations.

    container: ("box", side) -> centres uniform in [0, side]^3 (cells may
    protrude); ("cylinder", radius, length) -> bounding sphere inside the
    cylinder x^2 + y^2 <= radius^2, 0 <= z <= length.
    """
    p0, w0, n0 = evans_fung_surface(order)
    Rb = float(np.max(np.linalg.norm(p0, axis=0)))            # bounding-sphere radius
    if container[0] == "box":
        side = float(container[1])
        cent, tries = rsa_centres(rng, n_cells, Rb, [0, 0, 0], [side] * 3)
        cvol = side ** 3
    elif container[0] == "cylinder":
        rad, length = float(container[1]), float(container[2])
        rmax = rad - Rb
        cent, tries = rsa_centres(
            rng, n_cells, Rb, [-rmax, -rmax, Rb], [rmax, rmax, length - Rb],
            inside=lambda c: c[:, 0] ** 2 + c[:, 1] ** 2 <= rmax * rmax)
        cvol = math.pi * rad * rad * length
    else:
        raise ValueError(container)
    rots = random_rotations(rng, n_cells)
    npc = p0.shape[1]
    pos = np.einsum("cij,jn->icn", rots, p0) + cent.T[:, :, None]   # (3, cells, npc)
    nrm = np.einsum("cij,jn->icn", rots, n0)
    area = float(w0.sum())
    cell_vol = evans_fung_volume()
    return PointSet(
        pos=np.ascontiguousarray(pos.reshape(3, -1)),
        weight=np.tile(w0, n_cells),
        normal=np.ascontiguousarray(nrm.reshape(3, -1)),
        group=np.repeat(np.arange(n_cells, dtype=np.int32), npc),
        group_h=np.full(n_cells, math.sqrt(area / npc)),
        meta=dict(kind="cells", n_cells=n_cells, points_per_cell=npc, rsa_tries=int(tries),
                  bounding_radius=Rb, cell_area=area, cell_volume=cell_vol,
                  cell_volume_fraction=n_cells * cell_vol / cvol,
                  sphere_volume_fraction=n_cells * 4.0 / 3.0 * math.pi * Rb ** 3 / cvol,
                  centres=cent, container=container))


def cylinder_wall(radius=50.0, length=400.0, n_theta=64, n_z=64, q=16):
    """Open cylinder x^2+y^2 = radius^2, 0 <= z <= length (lateral surface only).

    n_theta x n_z patches, each with q x q Gauss-Legendre nodes on the exact
    cylinder map; weight w = w_i w_j (dtheta/2)(dz/2) radius; outward normal
    (cos theta, sin theta, 0).  Points are patch-major (q*q per patch)."""
    t, wt = np.polynomial.legendre.leggauss(q)
    dth, dz = 2 * np.pi / n_theta, length / n_z
    pi_, pj = np.meshgrid(np.arange(n_theta), np.arange(n_z), indexing="ij")
    pi_, pj = pi_.reshape(-1), pj.reshape(-1)                    # patch index order
    ti, tj = np.meshgrid(t, t, indexing="ij")
    wi, wj = np.meshgrid(wt, wt, indexing="ij")
    th = (pi_[:, None] + 0.5) * dth + 0.5 * dth * ti.reshape(1, -1)
    zz = (pj[:, None] + 0.5) * dz + 0.5 * dz * tj.reshape(1, -1)
    w = (wi * wj).reshape(1, -1) * (0.5 * dth) * (0.5 * dz) * radius
    w = np.broadcast_to(w, th.shape)
    pos = np.stack([radius * np.cos(th), radius * np.sin(th), zz]).reshape(3, -1)
    nrm = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)]).reshape(3, -1)
    npatch = n_theta * n_z
    area_patch = dth * radius * dz
    return PointSet(pos=np.ascontiguousarray(pos), weight=np.ascontiguousarray(w.reshape(-1)),
                    normal=np.ascontiguousarray(nrm),
                    group=np.repeat(np.arange(npatch, dtype=np.int32), q * q),
                    group_h=np.full(npatch, math.sqrt(area_patch / (q * q))),
                    meta=dict(kind="wall", radius=radius, length=length, n_patches=npatch,
                              points_per_patch=q * q, q=q, nodes_1d=t, weights_1d=wt))


# Cube faces as (outward axis, first tangent, second tangent) with t1 x t2 = axis,
# so that X_u x X_v of every patch points out of the surface.
_CUBE_FACES = (((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((-1, 0, 0), (0, 0, 1), (0, 1, 0)),
               ((0, 1, 0), (0, 0, 1), (1, 0, 0)), ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
               ((0, 0, 1), (1, 0, 0), (0, 1, 0)), ((0, 0, -1), (0, 1, 0), (1, 0, 0)))


def cube_sphere(radius=1.0, m=2, q=16, axes=(1.0, 1.0, 1.0), centre=(0.0, 0.0, 0.0), rule=None):
    """Closed patch surface: a sphere (or, with unequal `axes`, an ellipsoid)
    covered by 6 m^2 tensor-product patches.

    Each face of the cube [-1, 1]^3 is split into m x m squares and mapped to
    the sphere by the equiangular gnomonic map g = e + tan(pi a/4) t1 +
    tan(pi b/4) t2, X = centre + radius * axes * g/|g|.  Every patch carries
    q x q Gauss-Legendre nodes in its own parameter square [-1, 1]^2 (u along
    t1, v along t2, node k = i*q + j at (t_i, t_j)); weight w = w_i w_j
    |X_u x X_v| and unit normal X_u x X_v / |X_u x X_v|, both from the exact
    map, the normal outward.  Points are patch-major (q*q per patch).  `rule`
    = (nodes, weights) replaces the Gauss-Legendre rule (q is then its length)."""
    if rule is None:
        t, wt = np.polynomial.legendre.leggauss(q)
    else:
        t, wt = (np.asarray(a, dtype=np.float64) for a in rule)
        q = len(t)
    S = np.asarray(axes, dtype=np.float64)[:, None]
    ti, tj = [a.reshape(-1) for a in np.meshgrid(t, t, indexing="ij")]
    wij = np.outer(wt, wt).reshape(-1)
    pos, nrm, wts = [], [], []
    for e, t1, t2 in _CUBE_FACES:
        e, t1, t2 = (np.asarray(v, dtype=np.float64)[:, None] for v in (e, t1, t2))
        for a in range(m):
            for b in range(m):
                al = 0.25 * np.pi * (-1.0 + (2 * a + 1 + ti) / m)
                be = 0.25 * np.pi * (-1.0 + (2 * b + 1 + tj) / m)
                g = e + np.tan(al) * t1 + np.tan(be) * t2
                gn = np.linalg.norm(g, axis=0)
                gh = g / gn
                gu = (0.25 * np.pi / m) / np.cos(al) ** 2 * t1
                gv = (0.25 * np.pi / m) / np.cos(be) ** 2 * t2
                Xu = radius * S * (gu - gh * (gh * gu).sum(0)) / gn
                Xv = radius * S * (gv - gh * (gh * gv).sum(0)) / gn
                c = np.cross(Xu, Xv, axis=0)
                cn = np.linalg.norm(c, axis=0)
                pos.append(np.asarray(centre, dtype=np.float64)[:, None] + radius * S * gh)
                nrm.append(c / cn)
                wts.append(wij * cn)
    npatch = 6 * m * m
    w = np.concatenate(wts)
    area = w.reshape(npatch, q * q).sum(1)
    return PointSet(pos=np.ascontiguousarray(np.concatenate(pos, axis=1)), weight=w,
                    normal=np.ascontiguousarray(np.concatenate(nrm, axis=1)),
                    group=np.repeat(np.arange(npatch, dtype=np.int32), q * q),
                    group_h=np.sqrt(area / (q * q)),
                    meta=dict(kind="cube_sphere", radius=radius, axes=tuple(axes), n_patches=npatch,
                              points_per_patch=q * q, q=q, nodes_1d=t, weights_1d=wt))


def cells_after_step(rng, cells, max_shift=0.5, max_angle=0.05):
    """Positions of the cells' points one time step later: each cell (a group)
    moves rigidly by a uniform random shift of at most max_shift per axis and a
    rotation by at most max_angle radians about its centroid.  Returns (3, N)."""
    x1 = np.empty_like(cells.pos)
    for g in np.unique(cells.group):
        idx = np.nonzero(cells.group == g)[0]
        c = cells.pos[:, idx].mean(axis=1, keepdims=True)
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        ang = rng.uniform(-max_angle, max_angle)
        K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
        Rm = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
        x1[:, idx] = c + Rm @ (cells.pos[:, idx] - c) + rng.uniform(-max_shift, max_shift, (3, 1))
    return x1


def group_offsets(group):
    """CSR offsets (n_groups + 1,) of points sorted by group id."""
    counts = np.bincount(np.asarray(group), minlength=int(np.max(group)) + 1 if len(group) else 0)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


# ----------------------------------------------------------------------------
# Octree leaves and interaction lists (FMM near field)
# ----------------------------------------------------------------------------
def clenshaw_curtis(q):
    """q-point Clenshaw-Curtis rule on [-1, 1]: nodes -cos(pi j / (q - 1)) in
    increasing order, weights from the moment equations sum_j w_j t_j^k =
    int_{-1}^{1} t^k dt, k < q."""
    t = -np.cos(np.pi * np.arange(q) / (q - 1))
    t[np.abs(t) < 1e-15] = 0.0
    k = np.arange(q)
    moments = np.where(k % 2 == 0, 2.0 / (k + 1), 0.0)
    w = np.linalg.solve(np.vander(t, q, increasing=True).T, moments)
    return t, w


def _spread_bits(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_keys(pos, lo, side, depth=21):
    """63-bit Morton keys of points in the cube [lo, lo+side]^3 at the given depth."""
    scale = (1 << depth) / side
    ij = np.clip(np.floor((pos - np.asarray(lo)[:, None]) * scale), 0, (1 << depth) - 1).astype(np.uint64)
    return (_spread_bits(ij[0]) << np.uint64(2)) | (_spread_bits(ij[1]) << np.uint64(1)) | _spread_bits(ij[2])


@dataclass
class Octree:
    perm: np.ndarray           # (N,) original index of the i-th sorted point
    leaf_ofs: np.ndarray       # (n_leaves+1,) int64 point offsets of each leaf (sorted order)
    leaf_level: np.ndarray     # (n_leaves,) int32
    leaf_centre: np.ndarray    # (n_leaves, 3)
    leaf_side: np.ndarray      # (n_leaves,)
    leaf_key: np.ndarray       # (n_leaves,) uint64 first Morton key of each leaf box


def build_octree(pos, lo, side, max_leaf=256, depth=21):
    """Adaptive octree: split a box while it holds more than max_leaf points.

    Points are sorted by Morton key; empty boxes are dropped; leaves come out
    in Morton order and partition the sorted points contiguously."""
    keys = morton_keys(pos, lo, side, depth)
    perm = np.argsort(keys, kind="stable")
    sk = keys[perm]
    n = len(sk)
    leaves = []                                   # (start, end, level, prefix)
    active = [(0, n, 0, 0)]
    while active:
        nxt = []
        for (s, e, lev, pre) in active:
            if e - s <= max_leaf or lev == depth:
                if e > s:
                    leaves.append((s, e, lev, pre))
                continue
            shift = np.uint64(3 * (depth - lev - 1))
            bounds = [(np.uint64(pre) * np.uint64(8) + np.uint64(c)) << shift for c in range(9)]
            idx = np.searchsorted(sk[s:e], np.array(bounds, dtype=np.uint64)) + s
            for c in range(8):
                if idx[c + 1] > idx[c]:
                    nxt.append((int(idx[c]), int(idx[c + 1]), lev + 1, pre * 8 + c))
        active = nxt
    leaves.sort(key=lambda t: t[0])
    starts = np.array([l[0] for l in leaves] + [n], dtype=np.int64)
    levels = np.array([l[2] for l in leaves], dtype=np.int32)
    cents, sides, lkeys = [], [], []
    for (s, e, lev, pre) in leaves:
        sd = side / (1 << lev)
        # de-interleave the prefix into box coordinates
        ix = iy = iz = 0
        for b in range(lev):
            c = (pre >> (3 * (lev - 1 - b))) & 7
            ix = (ix << 1) | ((c >> 2) & 1)
            iy = (iy << 1) | ((c >> 1) & 1)
            iz = (iz << 1) | (c & 1)
        cents.append([lo[0] + (ix + 0.5) * sd, lo[1] + (iy + 0.5) * sd, lo[2] + (iz + 0.5) * sd])
        sides.append(sd)
        lkeys.append(pre << (3 * (depth - lev)))
    return Octree(perm=perm, leaf_ofs=starts, leaf_level=levels,
                  leaf_centre=np.array(cents), leaf_side=np.array(sides),
                  leaf_key=np.array(lkeys, dtype=np.uint64))


def nearest_leaf_lists(rng, tree, kmin=27, kmax=60):
    """Per-leaf interaction list: K ~ U{kmin..kmax} nearest non-empty leaves by
    centre distance, the leaf itself included, ties broken by Morton order.
    Returns (ulist_ofs int64 (n_leaves+1,), ulist int32)."""
    from scipy.spatial import cKDTree
    c = tree.leaf_centre
    nl = len(c)
    K = rng.integers(kmin, kmax + 1, size=nl)
    kq = min(nl, kmax + 20)
    kd = cKDTree(c)
    _, cand = kd.query(c, k=kq)
    cand = np.asarray(cand).reshape(nl, kq)
    lists = []
    for L in range(nl):
        cd = cand[L]
        d2 = ((c[cd] - c[L]) ** 2).sum(1)
        k = min(int(K[L]), nl)
        if kq < nl and d2.max() <= np.sort(d2)[k - 1]:
            # the k-th distance ties with the candidate horizon: take the full ball
            cd = np.array(sorted(kd.query_ball_point(c[L], math.sqrt(d2.max()) * (1 + 1e-12))))
            d2 = ((c[cd] - c[L]) ** 2).sum(1)
        order = np.lexsort((cd, d2))
        lists.append(np.sort(cd[order[:k]]).astype(np.int32))
    ofs = np.zeros(nl + 1, dtype=np.int64)
    ofs[1:] = np.cumsum([len(l) for l in lists])
    return ofs, np.concatenate(lists) if lists else np.zeros(0, np.int32)


# ----------------------------------------------------------------------------
# Configurations (the five workload shapes)
# ----------------------------------------------------------------------------
CONFIG_SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}


def _densities(rng, n):
    return rng.standard_normal((3, n))


def make_config(k, seed=None):
    """Build workload k (1..5).  Returns a dict of NumPy arrays and metadata.

    1: 8 cells in a 30^3 box, SL, all points are sources and targets.
    2: 512 cells in a 120^3 box (278,528 points), SL.
    3: 128 cells in a 75.6^3 box (69,632 points), SL + adjoint of
       L = 0.5 |u - u_ref|^2.
    4: 3,840 cells in a cylinder (radius 50, length 400), octree leaves of at
       most 256 points and per-leaf lists of 27..60 nearest leaves, SL P2P.
    5: cylinder wall (1,048,576 points) double layer onto 960 cells
       (522,240 points), plus the cell-to-cell single layer, with adjoint.
    """
    seed = CONFIG_SEEDS[k] if seed is None else seed
    rng = np.random.default_rng(seed)
    out = dict(config=k, seed=seed)
    if k in (1, 2, 3):
        n_cells, side = {1: (8, 30.0), 2: (512, 120.0), 3: (128, 75.6)}[k]
        cells = place_cells(rng, n_cells, ("box", side))
        out["cells"] = cells
        out["f"] = _densities(rng, cells.n)
        if k == 3:
            out["u_ref"] = _densities(rng, cells.n)
    elif k == 4:
        cells = place_cells(rng, 3840, ("cylinder", 50.0, 400.0))
        lo = np.array([-200.0, -200.0, 0.0])
        tree = build_octree(cells.pos, lo, 400.0, max_leaf=256)
        p = tree.perm
        cells = PointSet(pos=np.ascontiguousarray(cells.pos[:, p]), weight=cells.weight[p].copy(),
                         normal=np.ascontiguousarray(cells.normal[:, p]), group=cells.group[p].copy(),
                         group_h=cells.group_h, meta=cells.meta)
        out["cells"] = cells
        out["tree"] = tree
        ofs, ul = nearest_leaf_lists(rng, tree)
        out["ulist_ofs"], out["ulist"] = ofs, ul
        out["f"] = _densities(rng, cells.n)
    elif k == 5:
        wall = cylinder_wall()
        cells = place_cells(rng, 960, ("cylinder", 50.0, 400.0))
        out["wall"], out["cells"] = wall, cells
        out["phi"] = _densities(rng, wall.n)
        out["f"] = _densities(rng, cells.n)
        out["u_ref"] = _densities(rng, cells.n)
    else:
        raise ValueError(f"unknown config {k}")
    return out


def subset(rng, n, m):
    """m distinct indices out of n, sorted (seeded target samples)."""
    m = min(n, m)
    return np.sort(rng.choice(n, size=m, replace=False))


def pair_count_direct(group_src, group_trg, exclude_same_group=True):
    """Number of (target, source) pairs the direct sum evaluates, counting
    only the group rule (coincident points are not expected in these inputs)."""
    ns, nt = len(group_src), len(group_trg)
    if not exclude_same_group:
        return ns * nt
    gs = np.bincount(group_src)
    gt = np.bincount(group_trg, minlength=len(gs))
    m = min(len(gs), len(gt))
    return int(ns * nt - (gs[:m].astype(np.int64) * gt[:m]).sum())


def pair_count_p2p(leaf_ofs, ulist_ofs, ulist, group, exclude_same_group=True):
    """Number of (target, source) pairs a leaf-to-leaf sum evaluates when
    sources and targets are the same points in leaf order: for every leaf, its
    targets times the sources of its listed leaves, minus (same-group rule)
    the pairs whose two points carry the same group id.  Coincident points are
    not expected in these inputs."""
    import scipy.sparse as sp

    leaf_ofs = np.asarray(leaf_ofs, dtype=np.int64)
    ulist_ofs = np.asarray(ulist_ofs, dtype=np.int64)
    n_leaves = len(leaf_ofs) - 1
    size = np.diff(leaf_ofs)
    owner = np.repeat(np.arange(n_leaves), np.diff(ulist_ofs))
    listed = size[np.asarray(ulist, dtype=np.int64)]
    total = int((size[owner] * listed).sum())
    if not exclude_same_group:
        return total
    leaf_of_point = np.repeat(np.arange(n_leaves), size)
    g = np.asarray(group, dtype=np.int64)
    M = sp.csr_matrix((np.ones(len(g)), (leaf_of_point, g)), shape=(n_leaves, int(g.max()) + 1))
    A = sp.csr_matrix((np.ones(len(owner)), (owner, np.asarray(ulist, dtype=np.int64))),
                      shape=(n_leaves, n_leaves))
    same = M.multiply(A @ M).sum()
    return total - int(round(float(same)))
