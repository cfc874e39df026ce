// Internal declarations of the check-point (singular / near-singular)
// double-layer quadrature kernels.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stokes {

constexpr int kMaxQ = 24;     // nodes per patch side
constexpr int kMaxEta = 3;    // 4^eta sub-squares per patch
constexpr int kMaxP = 15;     // p + 1 check points per target

// The patch rule and the check-point parameters, passed by value to every
// kernel (about 0.4 KB of kernel arguments).
struct PatchRule {
    int32_t q, eta, p, pad;
    double R, r;              // first check point and spacing, fractions of L
    double t[kMaxQ], w[kMaxQ];
};

// Fine discretisation of every patch: positions, densities (U phi), weights
// and unit normals, patch-major with (2^eta q)^2 fine nodes per patch, and the
// patch sizes L = sqrt(sum of the patch's fine weights).
hipError_t launch_upsample(const PatchRule& rule, int64_t n_patches, const double* node_xyz,
                           const double* density, double* fine_xyz, double* fine_density,
                           double* fine_weight, double* fine_normal, double* patch_size,
                           hipStream_t stream);

// Check points c[t*(p+1) + i] = y_t - (R + i r) L n_t of every target.  With
// trg_patch == nullptr the targets are the patch nodes on the surface.
hipError_t launch_check_points(const PatchRule& rule, int64_t n_patches, const double* node_xyz,
                               const double* patch_size, int64_t n_trg, const int32_t* trg_patch,
                               const double* trg_uvd, double* check_xyz, hipStream_t stream);

// vel[t] (+)= sum_i e_i(d_t) check_vel[t*(p+1) + i].
hipError_t launch_extrapolate(const PatchRule& rule, int64_t n_patches, const double* patch_size,
                              int64_t n_trg, const int32_t* trg_patch, const double* trg_uvd,
                              const double* check_vel, double* vel, int accumulate,
                              hipStream_t stream);

}  // namespace stokes
