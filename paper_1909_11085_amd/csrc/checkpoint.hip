// Check-point quadrature of the double layer on and near a patched surface
// (Sec. 3.1, "Singular and near-singular integral quadrature"): the kernels
// around the direct double-layer sum.
//
//   upsample      every patch's degree-(q-1) tensor-product interpolant
//                 evaluated on the patch rule repeated over 4^eta sub-squares:
//                 fine positions, U phi, weights w_i w_j / 4^eta |X_u x X_v|
//                 and normals X_u x X_v / |X_u x X_v|.  One workgroup per
//                 sub-square; the contraction is separable (over v, then u)
//                 through LDS.
//   patch_size    L = sqrt(sum of a patch's fine weights), one wave per patch,
//                 fixed-order reduction.
//   check_points  y = P(u*, v*), n from X_u x X_v, c_i = y - (R + i r) L n.
//                 One wave per target; lanes run over the q*q node pairs.
//   extrapolate   u(x) = sum_i e_i u(c_i), e_i the Lagrange basis of the
//                 distances s_i = (R + i r) L evaluated at the target's d
//                 (eq. sing-quad).  One thread per target.
//
// The velocities at the check points (eq. quad_check_points) come from the
// direct double-layer sum with the fine nodes as sources.  Everything here is
// a few percent of that sum's time at most: the kernels are kept simple.
#include <math.h>

#include "checkpoint.hpp"
#include "common.hpp"

namespace stokes {
namespace {

constexpr int kCpBlock = 256;
constexpr int kCpWaves = kCpBlock / kWave;
constexpr int64_t kCpMaxGrid = 1 << 20;   // grid-stride loops beyond this many workgroups

unsigned cp_grid(int64_t units) { return (unsigned)(units < kCpMaxGrid ? units : kCpMaxGrid); }

// l_m(x) = prod_{k != m} (x - t_k) / (t_m - t_k) and its derivative, both
// carried along one pass over k: (P, P') <- (P f_k, P' f_k + P / (t_m - t_k)).
// At x = t_m every factor is exactly 1 and at x = t_k (k != m) one factor is
// exactly 0, so the basis is the identity at the nodes.
__device__ __forceinline__ void lagrange(const double* t, int q, int m, double x, double& v, double& dv) {
    const double tm = t[m];
    double P = 1.0, D = 0.0;
    for (int k = 0; k < q; ++k) {
        if (k == m) continue;
        const double den = tm - t[k];
        const double f = (x - t[k]) / den;
        D = D * f + P / den;
        P = P * f;
    }
    v = P;
    dv = D;
}

__device__ __forceinline__ void load_nodes(const PatchRule& R, double* s_t, double* s_w) {
    if (threadIdx.x == 0)
        for (int k = 0; k < R.q; ++k) {
            s_t[k] = R.t[k];
            if (s_w) s_w[k] = R.w[k];
        }
    __syncthreads();
}

// Dynamic LDS of upsample_kernel, in doubles: nodes, weights, four q x q basis
// tables and nine q x q partial contractions.
constexpr size_t upsample_lds_doubles(int q) { return 2 * kMaxQ + 13 * (size_t)q * q; }

__global__ __launch_bounds__(kCpBlock) void upsample_kernel(
    PatchRule R, int64_t n_nodes, const double* __restrict__ X, const double* __restrict__ F,
    double* __restrict__ fx, double* __restrict__ fphi, double* __restrict__ fw,
    double* __restrict__ fn, int64_t n_fine) {
    extern __shared__ double sh[];
    const int q = R.q, qq = q * q, ns = 1 << R.eta, nsq = ns * q;
    double* s_t = sh;
    double* s_w = s_t + kMaxQ;
    double* Bu = s_w + kMaxQ;     // Bu[i*q + m] = l_m(u_i), u_i the sub-square's i-th node
    double* Du = Bu + qq;
    double* Bv = Du + qq;         // Bv[j*q + l] = l_l(v_j)
    double* Dv = Bv + qq;
    double* T = Dv + qq;          // T[(c*q + m)*q + j], c = 0..8
    load_nodes(R, s_t, s_w);

    const int tid = threadIdx.x;
    const double inv_ns = 1.0 / ns;
    const int64_t n_blk = n_nodes / qq * ns * ns;
    for (int64_t blk = blockIdx.x; blk < n_blk; blk += gridDim.x) {    // uniform over the workgroup
        const int64_t patch = blk / (ns * ns);
        const int sub = (int)(blk % (ns * ns));
        const int au = sub / ns, av = sub % ns;

        for (int e = tid; e < qq; e += kCpBlock) {
            const int i = e / q, m = e % q;
            double v, dv;
            lagrange(s_t, q, m, -1.0 + (2 * au + 1 + s_t[i]) / ns, v, dv);
            Bu[e] = v;
            Du[e] = dv;
            lagrange(s_t, q, m, -1.0 + (2 * av + 1 + s_t[i]) / ns, v, dv);
            Bv[e] = v;
            Dv[e] = dv;
        }
        __syncthreads();

        // Contraction over the second patch index l:
        //   c = 0..2: X_c B_v,  c = 3..5: phi_c B_v (when phi is given),  c = 6..8: X_c D_v.
        const int64_t base = patch * qq;
        for (int e = tid; e < 9 * qq; e += kCpBlock) {
            const int c = e / qq, rem = e % qq, m = rem / q, j = rem % q;
            if (!F && c >= 3 && c < 6) continue;
            const double* src =
                (c < 3 ? X + c * n_nodes : c < 6 ? F + (c - 3) * n_nodes : X + (c - 6) * n_nodes) + base +
                (int64_t)m * q;
            const double* b = (c < 6 ? Bv : Dv) + j * q;
            double s = 0.0;
            for (int l = 0; l < q; ++l) s = fma(src[l], b[l], s);
            T[e] = s;
        }
        __syncthreads();

        // Contraction over the first index m, then normal and weight.
        for (int e = tid; e < qq; e += kCpBlock) {
            const int i = e / q, j = e % q;
            double pos[3] = {0.0, 0.0, 0.0}, phi[3] = {0.0, 0.0, 0.0};
            double xu[3] = {0.0, 0.0, 0.0}, xv[3] = {0.0, 0.0, 0.0};
            for (int m = 0; m < q; ++m) {
                const double bu = Bu[i * q + m], du = Du[i * q + m];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double tb = T[(c * q + m) * q + j];
                    pos[c] = fma(bu, tb, pos[c]);
                    xu[c] = fma(du, tb, xu[c]);
                    if (F) phi[c] = fma(bu, T[((c + 3) * q + m) * q + j], phi[c]);
                    xv[c] = fma(bu, T[((c + 6) * q + m) * q + j], xv[c]);
                }
            }
            const double nx = xu[1] * xv[2] - xu[2] * xv[1];
            const double ny = xu[2] * xv[0] - xu[0] * xv[2];
            const double nz = xu[0] * xv[1] - xu[1] * xv[0];
            const double a = sqrt(nx * nx + ny * ny + nz * nz);
            const int64_t k = patch * nsq * nsq + (int64_t)(au * q + i) * nsq + (av * q + j);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fx[c * n_fine + k] = pos[c];
                if (F) fphi[c * n_fine + k] = phi[c];
            }
            fn[k] = nx / a;
            fn[n_fine + k] = ny / a;
            fn[2 * n_fine + k] = nz / a;
            fw[k] = (s_w[i] * inv_ns) * (s_w[j] * inv_ns) * a;
        }
        __syncthreads();                          // tables and T are rewritten by the next sub-square
    }
}

__global__ __launch_bounds__(kCpBlock) void patch_size_kernel(const double* __restrict__ fw, int64_t n_patches,
                                                              int64_t per_patch, double* __restrict__ L) {
    const int lane = threadIdx.x % kWave;
    for (int64_t patch = (int64_t)blockIdx.x * kCpWaves + threadIdx.x / kWave; patch < n_patches;
         patch += (int64_t)gridDim.x * kCpWaves) {   // uniform over the wave
        const double* w = fw + patch * per_patch;
        double s = 0.0;
        for (int64_t k = lane; k < per_patch; k += kWave) s += w[k];
        for (int o = kWave / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) L[patch] = sqrt(s);
    }
}

// Target t: patch and (u, v), from the descriptor arrays or, without them, the
// t-th patch node.
__device__ __forceinline__ int64_t target_patch(int64_t t, int qq, const int32_t* trg_patch) {
    return trg_patch ? (int64_t)trg_patch[t] : t / qq;
}

__global__ __launch_bounds__(kCpBlock) void check_points_kernel(
    PatchRule R, int64_t n_patches, int64_t n_nodes, const double* __restrict__ X,
    const double* __restrict__ Lp, int64_t n_trg, const int32_t* __restrict__ trg_patch,
    const double* __restrict__ trg_uvd, double* __restrict__ cx, int64_t n_check) {
    __shared__ double s_t[kMaxQ];
    load_nodes(R, s_t, nullptr);
    const int q = R.q, qq = q * q, p1 = R.p + 1;
    const int lane = threadIdx.x % kWave;
    for (int64_t t = (int64_t)blockIdx.x * kCpWaves + threadIdx.x / kWave; t < n_trg;
         t += (int64_t)gridDim.x * kCpWaves) {     // uniform over the wave
        const int64_t patch = target_patch(t, qq, trg_patch);
        double u, v;
        if (trg_patch) {
            u = trg_uvd[t];
            v = trg_uvd[n_trg + t];
        } else {
            const int r = (int)(t % qq);
            u = s_t[r / q];
            v = s_t[r % q];
        }
        const bool bad = patch < 0 || patch >= n_patches;
        const int64_t pbase = (bad ? 0 : patch) * qq;

        // lanes 0..q-1 hold l_m(u), l_m'(u); lanes 32..32+q-1 hold l_l(v), l_l'(v)
        double b = 0.0, db = 0.0;
        if ((lane & 31) < q) lagrange(s_t, q, lane & 31, lane < 32 ? u : v, b, db);

        // y, X_u and X_v: sums over the q*q nodes (m, l), spread over the lanes
        double acc[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[c] = 0.0;
        for (int e0 = 0; e0 < qq; e0 += kWave) {    // uniform trip count: every lane shuffles
            const bool ok = e0 + lane < qq;
            const int e = ok ? e0 + lane : qq - 1;
            const int m = e / q, l = e % q;
            const double bu = __shfl(b, m), du = __shfl(db, m);
            const double bv = __shfl(b, 32 + l), dv = __shfl(db, 32 + l);
            if (ok) {
                const double w0 = bu * bv, wu = du * bv, wv = bu * dv;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double x = X[c * n_nodes + pbase + e];
                    acc[c] = fma(w0, x, acc[c]);
                    acc[3 + c] = fma(wu, x, acc[3 + c]);
                    acc[6 + c] = fma(wv, x, acc[6 + c]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 9; ++c)
            for (int o = kWave / 2; o >= 1; o >>= 1) acc[c] += __shfl_xor(acc[c], o);

        const double* xu = acc + 3;
        const double* xv = acc + 6;
        double n0 = xu[1] * xv[2] - xu[2] * xv[1];
        double n1 = xu[2] * xv[0] - xu[0] * xv[2];
        double n2 = xu[0] * xv[1] - xu[1] * xv[0];
        const double a = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        n0 /= a;
        n1 /= a;
        n2 /= a;
        if (lane < p1) {
            const double L = bad ? nan("") : Lp[bad ? 0 : patch];
            const double s = (R.R + R.r * lane) * L;
            const int64_t k = t * p1 + lane;
            cx[k] = acc[0] - s * n0;
            cx[n_check + k] = acc[1] - s * n1;
            cx[2 * n_check + k] = acc[2] - s * n2;
        }
    }
}

__global__ __launch_bounds__(kCpBlock) void extrapolate_kernel(
    PatchRule R, int64_t n_patches, const double* __restrict__ Lp, int64_t n_trg,
    const int32_t* __restrict__ trg_patch, const double* __restrict__ trg_uvd,
    const double* __restrict__ cv, int64_t n_check, double* __restrict__ vel, int accumulate) {
    const int q = R.q, p1 = R.p + 1;
    for (int64_t t = (int64_t)blockIdx.x * kCpBlock + threadIdx.x; t < n_trg;
         t += (int64_t)gridDim.x * kCpBlock) {
        const int64_t patch = target_patch(t, q * q, trg_patch);
        const bool bad = patch < 0 || patch >= n_patches;
        const double L = bad ? nan("") : Lp[bad ? 0 : patch];
        const double d = trg_patch ? trg_uvd[2 * n_trg + t] : 0.0;
        double u[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < p1; ++i) {
            const double si = (R.R + R.r * i) * L;
            double e = 1.0;
            for (int m = 0; m < p1; ++m) {
                if (m == i) continue;
                const double sm = (R.R + R.r * m) * L;
                e *= (d - sm) / (si - sm);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) u[c] = fma(e, cv[c * n_check + t * p1 + i], u[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) vel[c * n_trg + t] = accumulate ? vel[c * n_trg + t] + u[c] : u[c];
    }
}

}  // namespace

hipError_t launch_upsample(const PatchRule& rule, int64_t n_patches, const double* node_xyz,
                           const double* density, double* fine_xyz, double* fine_density,
                           double* fine_weight, double* fine_normal, double* patch_size,
                           hipStream_t stream) {
    if (n_patches <= 0) return hipSuccess;
    const int64_t qq = (int64_t)rule.q * rule.q, ns2 = (int64_t)1 << (2 * rule.eta);
    const int64_t n_nodes = n_patches * qq, per_patch = ns2 * qq, n_fine = n_patches * per_patch;
    const size_t lds = upsample_lds_doubles(rule.q) * sizeof(double);
    hipLaunchKernelGGL(upsample_kernel, dim3(cp_grid(n_patches * ns2)), dim3(kCpBlock), lds, stream, rule,
                       n_nodes, node_xyz, density, fine_xyz, fine_density, fine_weight, fine_normal, n_fine);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(patch_size_kernel, dim3(cp_grid(ceil_div(n_patches, kCpWaves))), dim3(kCpBlock), 0,
                       stream, fine_weight, n_patches, per_patch, patch_size);
    return hipGetLastError();
}

hipError_t launch_check_points(const PatchRule& rule, int64_t n_patches, const double* node_xyz,
                               const double* patch_size, int64_t n_trg, const int32_t* trg_patch,
                               const double* trg_uvd, double* check_xyz, hipStream_t stream) {
    if (n_trg <= 0) return hipSuccess;
    const int64_t n_nodes = n_patches * rule.q * rule.q;
    hipLaunchKernelGGL(check_points_kernel, dim3(cp_grid(ceil_div(n_trg, kCpWaves))), dim3(kCpBlock), 0, stream,
                       rule, n_patches, n_nodes, node_xyz, patch_size, n_trg, trg_patch, trg_uvd, check_xyz,
                       n_trg * (rule.p + 1));
    return hipGetLastError();
}

hipError_t launch_extrapolate(const PatchRule& rule, int64_t n_patches, const double* patch_size,
                              int64_t n_trg, const int32_t* trg_patch, const double* trg_uvd,
                              const double* check_vel, double* vel, int accumulate,
                              hipStream_t stream) {
    if (n_trg <= 0) return hipSuccess;
    hipLaunchKernelGGL(extrapolate_kernel, dim3(cp_grid(ceil_div(n_trg, kCpBlock))), dim3(kCpBlock), 0, stream,
                       rule, n_patches, patch_size, n_trg, trg_patch, trg_uvd, check_vel, n_trg * (rule.p + 1),
                       vel, accumulate);
    return hipGetLastError();
}

}  // namespace stokes
