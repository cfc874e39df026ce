// Internal declarations of the adjoint (vector-Jacobian product) sums.
#pragma once
#include "common.hpp"

namespace stokes {
size_t vjp_workspace_bytes(int kernel, int mixed, int64_t n_src, int64_t n_trg, int n_cu);
}  // namespace stokes
