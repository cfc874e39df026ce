"""MI355X-native (gfx950) Stokes kernel sums for boundary-integral red-blood-cell flow.

Single-layer (Stokeslet) and double-layer (stresslet) sums from surface
quadrature points to targets, in direct and leaf-to-leaf (FMM near-field)
form, in float64 or mixed float32/float64, with hand-written adjoints, and the
check-point quadrature of the double layer on and near a patched surface, as
hand-written HIP kernels behind the C ABI of ``include/stokes_mi355x.h``.

``workloads`` (seeded synthetic inputs) imports without torch; the compute
API (``sl``, ``dl``, ...) loads the HIP library on first use.
"""
_API = ("sl", "dl", "sl_vjp", "dl_vjp", "sl_diff", "dl_diff", "p2p_leaf", "p2p_sl_vjp", "p2p_dl_vjp", "p2p_diff", "P2PPlan",
        "context",
        "set_grid_override", "set_pair_symmetry", "debug_pair_classes", "StokesSL", "StokesDL", "StokesP2P",
        "timing_enable", "timing_read",
        "patch_upsample", "dl_checkpoint", "bie_apply", "bie_solve", "space_time_boxes",
        "collision_candidates", "FMMPlan", "fmm_sl", "fmm_dl")

__all__ = list(_API) + ["workloads"]


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
