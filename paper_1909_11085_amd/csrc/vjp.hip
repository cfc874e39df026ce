// Adjoint sums: not implemented yet in this revision.
#include "../../include/stokes_mi355x.h"
#include "vjp.hpp"

namespace stokes {
size_t vjp_workspace_bytes(int, int, int64_t, int64_t, int) { return 0; }
}  // namespace stokes

extern "C" {
int stokes_sl_vjp(stokes_ctx*, int64_t, const double*, const double*, const double*, int64_t,
                  const double*, double, const stokes_exclusion*, const stokes_opts*,
                  const double*, double*, double*, double*, void*, size_t, void*) {
    return STOKES_EUNSUPPORTED;
}
int stokes_dl_vjp(stokes_ctx*, int64_t, const double*, const double*, const double*,
                  const double*, int64_t, const double*, const stokes_exclusion*,
                  const stokes_opts*, const double*, double*, double*, double*, void*, size_t,
                  void*) {
    return STOKES_EUNSUPPORTED;
}
}
