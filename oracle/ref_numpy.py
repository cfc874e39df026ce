"""Tiny vectorised NumPy version of the oracle sums -- test infrastructure only.

A second, independent transcription of the same definitions (single layer,
eq. sl_stokes; double layer, after eq. double_layer_int_eq; weights times
densities, eq. smooth_double_layer_int_eq_patches_disc; the "other cells only"
rule of Sec. 2.2, step 1(d)), written over dense (targets x sources) arrays.
It exists to cross-check the C oracle's array layout and loop bounds on inputs
of at most a few hundred points; it is not a pin by itself.
"""
import numpy as np


def _pairs(src, trg, src_group, trg_group, exclude_same_group):
    r = trg.T[:, None, :] - src.T[None, :, :]                 # (nt, ns, 3)
    r2 = (r * r).sum(-1)
    keep = r2 > 0
    if exclude_same_group:
        keep &= np.asarray(trg_group)[:, None] != np.asarray(src_group)[None, :]
    rho = np.sqrt(np.where(keep, r2, 1.0))
    return r, rho, keep


def sl(src, f, w, trg, mu=1.0, src_group=None, trg_group=None, exclude_same_group=False):
    r, rho, keep = _pairs(src, trg, src_group, trg_group, exclude_same_group)
    q = (w[None, :] * f).T                                     # (ns, 3)
    rq = (r * q[None]).sum(-1)
    t = q[None] / rho[..., None] + r * (rq / rho ** 3)[..., None]
    t[~keep] = 0.0
    return (t.sum(1) / (8 * np.pi * mu)).T


def dl(src, phi, w, nrm, trg, src_group=None, trg_group=None, exclude_same_group=False):
    r, rho, keep = _pairs(src, trg, src_group, trg_group, exclude_same_group)
    q = (w[None, :] * phi).T
    rn = (r * nrm.T[None]).sum(-1)
    rq = (r * q[None]).sum(-1)
    t = r * (rn * rq / rho ** 5)[..., None]
    t[~keep] = 0.0
    return (t.sum(1) * 6.0 / (8 * np.pi)).T
