// Internal declarations of the kernel-independent FMM for the single- and
// double-layer sums (uniform octree).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

struct stokes_fmm_plan;

namespace stokes {

constexpr int kFmmMinOrder = 2, kFmmMaxOrder = 10;   // points per edge of the cube surfaces
constexpr int kFmmMinDepth = 2, kFmmMaxDepth = 7;

// Pseudo-inverse of a row-major n x n matrix by one-sided Jacobi SVD,
// dropping singular values below rcond times the largest (host).
void pinv_jacobi(const std::vector<double>& K, int n, double rcond, std::vector<double>& P);

int fmm_plan_build(int device, int order, stokes_fmm_plan** plan, std::string& err);
void fmm_plan_free(stokes_fmm_plan* plan);
int fmm_plan_order(const stokes_fmm_plan* plan);
int fmm_plan_device(const stokes_fmm_plan* plan);

struct FmmInputs {
    int64_t n_src, n_trg;
    const double* src_xyz;     // (3, n_src)
    const double* density;     // (3, n_src)
    const double* weight;      // (n_src)
    const double* normal;      // (3, n_src) for double-layer sources, else null
    const double* trg_xyz;     // (3, n_trg)
    double centre[3], half_width;
    int depth;
    double pref;               // 1 / (8 pi mu) (single layer) or 1 / (8 pi) (double layer)
    int accumulate;
    int mixed;                 // near-field pairs in float32
};

size_t fmm_workspace_bytes(int order, int64_t n_src, int64_t n_trg, int depth);

// Single layer when in.normal is null, double layer otherwise.
hipError_t launch_fmm(const stokes_fmm_plan* plan, const FmmInputs& in, double* out, void* ws, hipStream_t stream);

}  // namespace stokes
