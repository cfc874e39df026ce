// Internal declarations of the same-group correction of all-pairs sums.  Not
// part of the public C ABI.
#pragma once

#include "common.hpp"

namespace stokes {

// Workspace of launch_same_group_subtract (0 when there is nothing to do).
size_t same_group_workspace_bytes(int kernel, int64_t n_src, int64_t n_trg, int32_t n_groups);

// out(:, n) -= the sum over the sources of target n's group (rho = 0 skipped)
// of pref K(x_n - y_m) q_m, in float64; in.src_group, in.trg_group and
// in.n_groups > 0 are read, an id outside [0, n_groups) makes every output
// component NaN.  Asynchronous on `stream`.
hipError_t launch_same_group_subtract(const SumInputs& in, double* out, void* ws, hipStream_t stream);

}  // namespace stokes
