// Vector kernels of the boundary-integral solve: the dot products, linear
// combinations and scalings of GMRES's Arnoldi process (classical Gram-Schmidt
// applied twice).  All of them are HBM-bound streams over vectors of 3N
// doubles; the matrix-vector product (the check-point double-layer quadrature)
// dominates a solve by orders of magnitude.
//
// Reductions are two-stage with a fixed partition (a function of the length
// only) and fixed orders inside each stage, so results are reproducible.
#include <algorithm>

#include "bie.hpp"
#include "common.hpp"

namespace stokes {
namespace {

constexpr int kVecBlock = 256;
constexpr int64_t kVecMaxGrid = 1 << 16;

unsigned vec_grid(int64_t n) {
    const int64_t b = ceil_div(n, kVecBlock);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kVecMaxGrid));
}

__global__ __launch_bounds__(kVecBlock) void multi_dot_partial(const double* __restrict__ A, int64_t lda,
                                                               const double* __restrict__ b, int64_t n,
                                                               double* __restrict__ part) {
    __shared__ double red[kVecBlock];
    const int nblk = gridDim.x, j = blockIdx.y;
    const double* a = A + j * lda;
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBlock) s = fma(a[i], b[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kVecBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)j * nblk + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kVecBlock) void multi_dot_final(const double* __restrict__ part, int nblk, int nv,
                                                             double* __restrict__ out) {
    for (int j = threadIdx.x; j < nv; j += kVecBlock) {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += part[(int64_t)j * nblk + k];
        out[j] = s;
    }
}

template <bool SET>
__global__ __launch_bounds__(kVecBlock) void combo_kernel(double* __restrict__ w, const double* __restrict__ A,
                                                          int64_t lda, int nv, const double* __restrict__ coef,
                                                          int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecBlock) {
        double s = SET ? 0.0 : w[i];
        for (int j = 0; j < nv; ++j) s = SET ? fma(coef[j], A[j * lda + i], s) : fma(-coef[j], A[j * lda + i], s);
        w[i] = s;
    }
}

__global__ __launch_bounds__(kVecBlock) void scale_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                                          double s, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecBlock)
        dst[i] = s * src[i];
}

__global__ __launch_bounds__(kVecBlock) void weighted_normals_kernel(double* __restrict__ wn,
                                                                     const double* __restrict__ nrm,
                                                                     const double* __restrict__ w, int64_t n) {
    for (int64_t m = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; m < n; m += (int64_t)gridDim.x * kVecBlock)
#pragma unroll
        for (int c = 0; c < 3; ++c) wn[c * n + m] = w[m] * nrm[c * n + m];
}

}  // namespace

int reduce_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, ceil_div(n, 8192))); }

hipError_t launch_multi_dot(const double* A, int64_t lda, int nv, const double* b, int64_t n, double* part,
                            double* out, hipStream_t stream) {
    if (nv <= 0) return hipSuccess;
    const int nblk = reduce_blocks(n);
    hipLaunchKernelGGL(multi_dot_partial, dim3(nblk, nv), dim3(kVecBlock), 0, stream, A, lda, b, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(multi_dot_final, dim3(1), dim3(kVecBlock), 0, stream, part, nblk, nv, out);
    return hipGetLastError();
}

hipError_t launch_combo_sub(double* w, const double* A, int64_t lda, int nv, const double* coef, int64_t n,
                            hipStream_t stream) {
    if (nv <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(combo_kernel<false>, dim3(vec_grid(n)), dim3(kVecBlock), 0, stream, w, A, lda, nv, coef, n);
    return hipGetLastError();
}

hipError_t launch_combo_set(double* x, const double* A, int64_t lda, int nv, const double* coef, int64_t n,
                            hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(combo_kernel<true>, dim3(vec_grid(n)), dim3(kVecBlock), 0, stream, x, A, lda, nv, coef, n);
    return hipGetLastError();
}

hipError_t launch_scale(double* dst, const double* src, double s, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, dim3(vec_grid(n)), dim3(kVecBlock), 0, stream, dst, src, s, n);
    return hipGetLastError();
}

hipError_t launch_weighted_normals(double* wn, const double* normal, const double* weight, int64_t n_nodes,
                                   hipStream_t stream) {
    if (n_nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(weighted_normals_kernel, dim3(vec_grid(n_nodes)), dim3(kVecBlock), 0, stream, wn, normal,
                       weight, n_nodes);
    return hipGetLastError();
}

}  // namespace stokes
