// Internal declarations of the leaf-to-leaf (P2P) sums.
#pragma once
#include <string>

#include "common.hpp"

struct stokes_p2p_plan;

namespace stokes {

size_t p2p_workspace_bytes(int kernel, int mixed, int64_t n_src, int64_t n_trg, int32_t n_leaves);

// Validates the host leaf arrays and uploads the layout to the current device.
int p2p_plan_build(int device, int32_t n_leaves, int64_t n_src, int64_t n_trg,
                   const int64_t* src_ofs, const int64_t* trg_ofs, const int64_t* ulist_ofs,
                   const int32_t* ulist, int64_t n_ulist, stokes_p2p_plan** out, std::string& err);
void p2p_plan_free(stokes_p2p_plan* p);
// 0: n_src, 1: n_trg, 2: n_leaves, 3: pairs, 4: device
int64_t p2p_plan_info(const stokes_p2p_plan* p, int which);

hipError_t launch_p2p(const SumInputs& in, const stokes_p2p_plan* plan, double* out, int accumulate,
                      void* ws, hipStream_t stream, const KernelTimer& timer);

// The same sum from device leaf arrays, checked and cut into sorted work items
// on the device; malformed arrays make every output component NaN.  check =
// false skips the checks (layouts built by the library itself; n_ulist is then
// not used).
hipError_t launch_p2p_csr(const SumInputs& in, int32_t n_leaves, const int64_t* src_ofs, const int64_t* trg_ofs,
                          const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist, double* out,
                          int accumulate, void* ws, hipStream_t stream, const KernelTimer& timer,
                          bool check = true, const int32_t* ext_status = nullptr);
// (ext_status, with check = false: the verdict of an earlier launch_p2p_check.)

// Clears *status and sets it when the device leaf arrays break the layout's
// rules (the checks of launch_p2p_csr).
hipError_t launch_p2p_check(int32_t n_leaves, const int64_t* src_ofs, const int64_t* trg_ofs,
                            const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_src, int64_t n_trg,
                            int64_t n_ulist, int32_t* status, hipStream_t stream);

// The transposed lists: leaf L' lists, in increasing order and with
// multiplicity, the leaves whose lists hold L' (n_ulist entries; offsets
// n_leaves + 1).  With *status set, every entry goes to leaf 0 (nothing
// outside the arrays is read).  Workspace p2p_transpose_bytes(n_ulist).
size_t p2p_transpose_bytes(int64_t n_ulist);

// Adjoint of the leaf-to-leaf sum (float64) of in.kernel (0 single layer, 1
// double layer): each output may be null; in holds the forward's inputs
// (density, weight, normal, pref, pair rule).  The device leaf arrays are
// checked; malformed ones make the outputs NaN.
size_t p2p_vjp_workspace_bytes(int kernel, int64_t n_src, int64_t n_trg, int32_t n_leaves, int64_t n_ulist);
hipError_t launch_p2p_vjp(const SumInputs& in, int32_t n_leaves, const int64_t* src_ofs, const int64_t* trg_ofs,
                          const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist, const double* grad_vel,
                          double* grad_density, double* grad_src, double* grad_trg, int accumulate, void* ws,
                          hipStream_t stream);
hipError_t launch_p2p_transpose(int32_t n_leaves, const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist,
                                const int32_t* status, int64_t* ulist_ofs_t, int32_t* ulist_t, void* ws,
                                hipStream_t stream);

}  // namespace stokes
