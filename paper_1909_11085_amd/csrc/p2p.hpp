// Internal declarations of the leaf-to-leaf (P2P) sums.
#pragma once
#include "common.hpp"

namespace stokes {
size_t p2p_workspace_bytes(int kernel, int mixed, int64_t n_src, int64_t n_trg, int32_t n_leaves);
}  // namespace stokes
