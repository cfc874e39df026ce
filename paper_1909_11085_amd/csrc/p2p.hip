// Leaf-to-leaf (P2P) sums: not implemented yet in this revision.
#include "../../include/stokes_mi355x.h"
#include "p2p.hpp"

namespace stokes {
size_t p2p_workspace_bytes(int, int, int64_t, int64_t, int32_t) { return 0; }
}  // namespace stokes

extern "C" {
int stokes_p2p_plan_create(stokes_ctx*, int32_t, int64_t, int64_t, const int64_t*, const int64_t*,
                           const int64_t*, const int32_t*, int64_t, stokes_p2p_plan** plan) {
    if (plan) *plan = nullptr;
    return STOKES_EUNSUPPORTED;
}
void stokes_p2p_plan_destroy(stokes_p2p_plan*) {}
int stokes_p2p_plan_pairs(const stokes_p2p_plan*, int64_t*) { return STOKES_EUNSUPPORTED; }
int stokes_p2p_leaf_eval(stokes_ctx*, const stokes_p2p_plan*, int32_t, int64_t, const double*,
                         const double*, const double*, const double*, int64_t, const double*,
                         double, const stokes_exclusion*, const stokes_opts*, double*, void*,
                         size_t, void*) {
    return STOKES_EUNSUPPORTED;
}
}
