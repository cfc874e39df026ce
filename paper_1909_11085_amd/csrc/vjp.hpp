// Internal declarations of the adjoint (vector-Jacobian product) sums.
#pragma once
#include "common.hpp"

namespace stokes {

struct VjpInputs {
    int64_t n_src, n_trg;
    const double* src_xyz;
    const double* density;
    const double* weight;
    const double* normal;      // double layer only
    const double* trg_xyz;
    const double* grad_vel;    // (3, n_trg)
    int excl;
    const int32_t* src_group;
    const int32_t* trg_group;
    double pref;               // 1/(8 pi mu) or 6/(8 pi)
    int accumulate;
    double* grad_density;      // (3, n_src) or null
    double* grad_src;          // (3, n_src) or null
    double* grad_trg;          // (3, n_trg) or null
};

constexpr int kVjpPasses = 8;

// Resident workgroups of the adjoint pass kernels on a device with n_cu
// compute units (current device).
void vjp_resident(int n_cu, int out[kVjpPasses]);

// Workspace bytes of an adjoint call (kernel 0 = single, 1 = double layer):
// the largest of the passes it may run (passes run one after another).
size_t vjp_workspace_bytes(int kernel, int64_t n_src, int64_t n_trg, const int resident[kVjpPasses]);

// fused: shared point set with one combined position gradient (grad_src ==
// grad_trg), one pass.  Requires n_src, n_trg > 0.
hipError_t launch_sl_vjp(const VjpInputs& in, const int resident[kVjpPasses], bool fused, void* ws,
                         hipStream_t stream);
// combined: grad_src == grad_trg on a shared point set; the array receives
// the total position gradient (target pass, then the source pass adds).
hipError_t launch_dl_vjp(const VjpInputs& in, const int resident[kVjpPasses], bool combined, void* ws,
                         hipStream_t stream);

}  // namespace stokes
