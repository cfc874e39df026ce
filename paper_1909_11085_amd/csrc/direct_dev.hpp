// Device helpers of the direct (all-pairs) sums, shared by the one-sided
// kernels (direct.hip) and the each-pair-once kernels of shared point sets
// (sym.hip): wave reductions, target loading, the sub-tile near tests and the
// pair functions.  Internal, not part of the C ABI.
#pragma once
#include <float.h>
#include <limits.h>

#include "common.hpp"

namespace stokes {

// ---------------------------------------------------------------------------
// wave-level reductions (wave64, butterfly over lanes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_mini(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_maxi(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// 1/rho in float64 from A = 4 rho^2 (coordinates stored doubled, exactly):
// hardware estimate z ~ 1/sqrt(A) = 1/(2 rho) (about 24 correct bits,
// measured) and one Newton step, written as z (3 - A z^2) = 2 z (1.5 - A z^2/2)
// so that the factor 2 comes for free: three operations, ~1e-15 relative.
__device__ __forceinline__ double rinv_doubled(double A, bool skip) {
    const double z = skip ? 0.0 : __builtin_amdgcn_rsq(A);
    const double t = A * z;
    return z * __builtin_fma(-t, z, 3.0);
}

// ---------------------------------------------------------------------------
// target setup shared by both precisions
// ---------------------------------------------------------------------------
struct Box {
    double lo[3], hi[3];
    int32_t gmin, gmax;
    int32_t pad[2];
};

template <int T>
struct Targets {
    double x[T], y[T], z[T];
    int32_t g[T];
};

// Loads the wave's targets (T per lane: target tb + k*64 + lane) and returns
// the box and group range of the whole wave.  Lanes past n_trg load the last
// target (a real point, so the box stays conservative) and store nothing.
template <int T>
__device__ __forceinline__ Box load_targets(const SumInputs& in, int64_t tb, int lane,
                                            Targets<T>& t) {
    const int64_t n = in.n_trg;
    Box w;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    int gmn = INT_MAX, gmx = INT_MIN;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t idx = tb + (int64_t)k * kWave + lane;
        const int64_t ic = idx < n ? idx : n - 1;
        t.x[k] = in.trg_xyz[ic];
        t.y[k] = in.trg_xyz[n + ic];
        t.z[k] = in.trg_xyz[2 * n + ic];
        t.g[k] = in.trg_group ? in.trg_group[ic] : 0;
        lo[0] = fmin(lo[0], t.x[k]); hi[0] = fmax(hi[0], t.x[k]);
        lo[1] = fmin(lo[1], t.y[k]); hi[1] = fmax(hi[1], t.y[k]);
        lo[2] = fmin(lo[2], t.z[k]); hi[2] = fmax(hi[2], t.z[k]);
        gmn = min(gmn, t.g[k]);
        gmx = max(gmx, t.g[k]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) { w.lo[c] = wave_min(lo[c]); w.hi[c] = wave_max(hi[c]); }
    w.gmin = wave_mini(gmn);
    w.gmax = wave_maxi(gmx);
    w.pad[0] = w.pad[1] = 0;
    return w;
}

__device__ __forceinline__ double box_gap2(const Box& b, const SubMeta& m) {
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g = fmax(fmax(m.lo[c] - b.hi[c], b.lo[c] - m.hi[c]), 0.0);
        d2 = __builtin_fma(g, g, d2);
    }
    return d2;
}

__device__ __forceinline__ bool groups_overlap(const Box& b, const SubMeta& m) {
    return !(m.gmax < b.gmin || m.gmin > b.gmax);
}

// Squared distance from the near-pass boundary of a sub-tile.
//   FP64: only coincident points need care, so the limit is 0 (any overlap).
//   Mixed: pairs within the largest near radius (with slack for float32
//   rounding of the offsets, 2^-20 of the coordinate scale) take float64, and
//   pairs closer than an eighth of the sub-tile's extent e take the high + low
//   float32 offsets.  Beyond that, offsets from the sub-tile centre (at most
//   rho + e sqrt(3)/2 and e sqrt(3)/2) give each component of r to within
//   eps32 (1 + sqrt(3) e / (2 rho)) <= 8 eps32 relative.
template <bool MIXED>
__device__ __forceinline__ double near_limit2(const Box& w, const SubMeta& m) {
    if constexpr (!MIXED) {
        return 1e-200;
    } else {
        const double sext = fmax(fmax(m.hi[0] - m.lo[0], m.hi[1] - m.lo[1]), m.hi[2] - m.lo[2]);
        const double wext = fmax(fmax(w.hi[0] - w.lo[0], w.hi[1] - w.lo[1]), w.hi[2] - w.lo[2]);
        double cd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) cd += fabs(0.5 * (w.lo[c] + w.hi[c]) - m.ctr[c]);
        const double slack = 0x1p-20 * (cd + wext + sext);
        const double lim = fmax(__builtin_fma(1.001, m.rnear, slack), 0.125 * sext);
        return lim * lim;
    }
}

// Decides, uniformly for the wave, whether a sub-tile goes to the near pass:
// some target of the wave shares a group id with the sub-tile's range, or
// lies within the limit of its box.  The whole-wave box settles most
// sub-tiles before the per-target test.
template <int T, bool MIXED>
__device__ __forceinline__ bool needs_near(const Box& w, const Targets<T>& t, const SubMeta& m,
                                           bool excl) {
    const double lim2 = near_limit2<MIXED>(w, m);
    const bool wave_near = (excl && groups_overlap(w, m)) || !(box_gap2(w, m) > lim2);
    if (!wave_near) return false;
    bool any = false;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const double p[3] = {t.x[k], t.y[k], t.z[k]};
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double g = fmax(fmax(m.lo[c] - p[c], p[c] - m.hi[c]), 0.0);
            d2 = __builtin_fma(g, g, d2);
        }
        any |= (excl && t.g[k] >= m.gmin && t.g[k] <= m.gmax) || !(d2 > lim2);
    }
    return __ballot(any) != 0;
}

// Workgroup b of G processes units [b*U/G, (b+1)*U/G); the workgroup holding
// unit u is floor(((u+1)*G - 1)/U).
__device__ __forceinline__ int64_t unit_begin(int64_t b, int64_t U, int64_t G) { return b * U / G; }
__device__ __forceinline__ int64_t unit_owner(int64_t u, int64_t U, int64_t G) {
    return ((u + 1) * G - 1) / U;
}

// ---------------------------------------------------------------------------
// FP64 pair kernels (bare, without prefactor)
// ---------------------------------------------------------------------------
// Both points come in doubled, r' = 2r, and ri = 1/rho (see rinv_doubled):
//   single layer: (4q + r' (r'.q)/rho^2)/rho = 4 [q/rho + r (r.q)/rho^3]
//   double layer: r' (r'.n)(r'.q)/rho^5     = 8 r (r.n)(r.q)/rho^5
// The factors 4 and 8 are divided out of the prefactor after the sum.
template <int KT, bool MASKED>
__device__ __forceinline__ void pair_f64(const typename SrcRec<KT, 0>::type& s, double x, double y,
                                         double z, bool skip_group, double& ax, double& ay,
                                         double& az) {
    const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
    const double A = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double ri = rinv_doubled(A, MASKED && (skip_group || A == 0.0));
    const double ri2 = ri * ri;
    const double rq = __builtin_fma(dx, s.qx, __builtin_fma(dy, s.qy, dz * s.qz));
    if constexpr (KT == 0) {
        const double c = rq * ri2;
        ax = __builtin_fma(__builtin_fma(c, dx, s.q4x), ri, ax);
        ay = __builtin_fma(__builtin_fma(c, dy, s.q4y), ri, ay);
        az = __builtin_fma(__builtin_fma(c, dz, s.q4z), ri, az);
    } else {
        const double rn = __builtin_fma(dx, s.nx, __builtin_fma(dy, s.ny, dz * s.nz));
        const double c = rn * rq * (ri2 * ri2 * ri);
        ax = __builtin_fma(c, dx, ax);
        ay = __builtin_fma(c, dy, ay);
        az = __builtin_fma(c, dz, az);
    }
}

// Doubles a wave's target coordinates and box (exact), to match the FP64
// source records.
template <int T>
__device__ __forceinline__ void double_targets(Targets<T>& t, Box* w) {
#pragma unroll
    for (int k = 0; k < T; ++k) {
        t.x[k] *= 2.0;
        t.y[k] *= 2.0;
        t.z[k] *= 2.0;
    }
    if (w) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w->lo[c] *= 2.0;
            w->hi[c] *= 2.0;
        }
    }
}

// Iterates the flagged sub-tiles of one wave's flag row (64 flag bytes are
// read per step, one per lane); the near pass splits each row into
// kNearSlices interleaved slices, one per grid row, for balance.
constexpr int kNearSlices = 4;
template <typename F>
__device__ __forceinline__ void for_each_flagged(const uint8_t* fl, int64_t C, int lane, int slice,
                                                 F&& fn) {
    int n = 0;                                 // flagged sub-tiles seen so far (uniform)
    for (int64_t c0 = 0; c0 < C; c0 += kWave) {
        const uint32_t mine = (c0 + lane < C) ? fl[c0 + lane] : 0u;
        uint64_t nz = __ballot(mine != 0);
        while (nz) {
            const int l = __builtin_ctzll(nz);
            nz &= nz - 1;
            uint32_t f = (uint32_t)__builtin_amdgcn_readlane((int)mine, l);
            while (f) {
                const int s = __builtin_ctz(f);
                f &= f - 1;
                if (n++ % kNearSlices == slice) fn((c0 + l) * 4 + s);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Mixed precision: float32 pairs on centred offsets, float64 near pairs & sums
// ---------------------------------------------------------------------------
template <int KT>
__device__ __forceinline__ void pair_f32(const typename SrcRec<KT, 1>::type& s, float dx, float dy,
                                         float dz, bool skip, bool masked, float& ax, float& ay,
                                         float& az) {
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float ri = masked ? (skip ? 0.0f : __builtin_amdgcn_rsqf(r2)) : __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float rq = __builtin_fmaf(dx, s.qx, __builtin_fmaf(dy, s.qy, dz * s.qz));
    if constexpr (KT == 0) {
        const float c = rq * ri2;
        ax = __builtin_fmaf(__builtin_fmaf(c, dx, s.qx), ri, ax);
        ay = __builtin_fmaf(__builtin_fmaf(c, dy, s.qy), ri, ay);
        az = __builtin_fmaf(__builtin_fmaf(c, dz, s.qz), ri, az);
    } else {
        const float rn = __builtin_fmaf(dx, s.nx, __builtin_fmaf(dy, s.ny, dz * s.nz));
        const float c = rn * rq * (ri2 * ri2 * ri);
        ax = __builtin_fmaf(c, dx, ax);
        ay = __builtin_fmaf(c, dy, ay);
        az = __builtin_fmaf(c, dz, az);
    }
}

// One pair in float64 from the caller's arrays (near pairs of the mixed path).
template <int KT>
__device__ __forceinline__ void near_pair_f64(const SumInputs& in, int64_t m, double x, double y,
                                              double z, double& ax, double& ay, double& az) {
    const int64_t ns = in.n_src;
    const double dx = x - in.src_xyz[m];
    const double dy = y - in.src_xyz[ns + m];
    const double dz = z - in.src_xyz[2 * ns + m];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;
    const double w = in.weight[m];
    const double qx = w * in.density[m], qy = w * in.density[ns + m], qz = w * in.density[2 * ns + m];
    const double ri = 1.0 / sqrt(r2);
    const double rq = dx * qx + dy * qy + dz * qz;
    if constexpr (KT == 0) {
        const double c = rq * ri * ri;
        ax += (qx + c * dx) * ri;
        ay += (qy + c * dy) * ri;
        az += (qz + c * dz) * ri;
    } else {
        const double rn = dx * in.normal[m] + dy * in.normal[ns + m] + dz * in.normal[2 * ns + m];
        const double c = rn * rq * (ri * ri) * (ri * ri) * ri;
        ax += c * dx;
        ay += c * dy;
        az += c * dz;
    }
}

}  // namespace stokes
