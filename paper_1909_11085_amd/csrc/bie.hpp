// Internal declarations of the vector kernels of the boundary-integral solve
// (GMRES on the check-point double-layer operator).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stokes {

constexpr int kMaxKrylov = 100;   // GMRES iterations (basis vectors - 1) per solve

// Workgroups of the first reduction stage for vectors of n elements (a
// function of n only, so that sums are reproducible).
int reduce_blocks(int64_t n);

// out[j] = sum_i A[j*lda + i] * b[i] for j < nv, in a fixed order: per
// workgroup over its contiguous range, then over workgroups.  part holds
// nv * reduce_blocks(n) doubles.
hipError_t launch_multi_dot(const double* A, int64_t lda, int nv, const double* b, int64_t n,
                            double* part, double* out, hipStream_t stream);

// w[i] -= sum_j coef[j] * A[j*lda + i]  (coef in device memory).
hipError_t launch_combo_sub(double* w, const double* A, int64_t lda, int nv, const double* coef,
                            int64_t n, hipStream_t stream);

// x[i] = sum_j coef[j] * A[j*lda + i]  (coef in device memory).
hipError_t launch_combo_set(double* x, const double* A, int64_t lda, int nv, const double* coef,
                            int64_t n, hipStream_t stream);

// dst[i] = s * src[i].
hipError_t launch_scale(double* dst, const double* src, double s, int64_t n, hipStream_t stream);

// wn[c*N + m] = weight[m] * normal[c*N + m].
hipError_t launch_weighted_normals(double* wn, const double* normal, const double* weight, int64_t n_nodes,
                                   hipStream_t stream);

}  // namespace stokes
