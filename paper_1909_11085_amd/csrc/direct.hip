// Direct (all-pairs) Stokes kernel sums on gfx950.
//
// Single layer (Stokeslet, paper eq. sl_stokes) and double layer (stresslet,
// stated after eq. double_layer_int_eq), summed over the smooth quadrature of
// eq. smooth_double_layer_int_eq_patches_disc (strength q = w * density),
// with the "other cells only" rule of the explicit step (Sec. 3.2, step 1d)
// and distance-0 pairs skipped.
//
// Design (CDNA4, wave64):
//   * prep: one thread per source packs {position, q[, normal]} into a padded
//     record array and each wave summarises its 64-source sub-tile (bounding
//     box, group range, near radius).
//   * sum: a workgroup of 4 waves owns 4*64*T targets (T per lane, kept in
//     registers) and one split of the sources.  Sources stream through LDS
//     in steps of 256 records (register prefetch of the next step); every
//     lane of a wave reads the same record, a broadcast LDS read.
//   * per 64-source sub-tile the wave decides, uniformly, between a fast loop
//     with no per-pair tests (box far from the wave's targets and no shared
//     group) and a masked loop.  Mixed precision evaluates pairs in float32
//     on offsets from the sub-tile centre (each rounded once from float64),
//     sums each sub-tile in float32 and adds it into float64 accumulators.
//     In a close sub-tile (possible exclusions or near pairs, or a gap below
//     half the boxes' extents) r is formed from float32 high parts plus
//     float32 residues, and pairs within the near radius go through a float64
//     branch instead.
//   * several source splits write float64 partial sums that a second kernel
//     adds in fixed order (deterministic; no atomics).
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

// 1/sqrt(r2) in float64: hardware estimate (about 24 correct bits, measured)
// plus one Newton step y <- y + y (1 - r2 y^2)/2, leaving ~1e-15 relative.
__device__ __forceinline__ double rsqrt_nr(double r2) {
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    return __builtin_fma(0.5 * y0, e, y0);
}
__device__ __forceinline__ double rsqrt_nr_masked(double r2, bool skip) {
    const double y0 = skip ? 0.0 : __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    return __builtin_fma(0.5 * y0, e, y0);
}

struct DirectArgs {
    SumInputs in;
    const void* rec;          // packed source records
    const void* aux;          // FP64 path: padded int32 groups; mixed: float4 low parts
    const SubMeta* meta;
    int64_t n_sub, subs_per_split;
    double* out;              // final output when splits == 1, else partials
    int splits, accumulate;
};

// ---------------------------------------------------------------------------
// source prep
// ---------------------------------------------------------------------------
template <int KT, int MIXED>
__global__ __launch_bounds__(kBlock) void prep_sources(SumInputs in, void* rec_out, void* aux_out,
                                                       SubMeta* meta) {
    using Rec = typename SrcRec<KT, MIXED>::type;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;   // grid covers n_src_pad exactly
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n = in.n_src;
    const bool valid = i < n;
    double y[3] = {kPadPos, kPadPos, kPadPos}, q[3] = {0, 0, 0}, nv[3] = {0, 0, 0};
    double rn = 0.0;
    int32_t g = INT_MIN;
    if (valid) {
        const double w = in.weight[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            y[c] = in.src_xyz[c * n + i];
            q[c] = w * in.density[c * n + i];
            if (KT == 1) nv[c] = in.normal[c * n + i];
        }
        g = in.src_group ? in.src_group[i] : 0;
        if (MIXED && in.group_h) {
            if (g >= 0 && g < in.n_groups) {
                rn = in.near_frac * in.group_h[g];
            } else {   // invalid group id: poison this source's strength
                q[0] = q[1] = q[2] = __builtin_nan("");
            }
        }
    }
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = wave_min(valid ? y[c] : DBL_MAX);
        hi[c] = wave_max(valid ? y[c] : -DBL_MAX);
    }
    const int gmin = wave_mini(valid ? g : INT_MAX);
    const int gmax = wave_maxi(valid ? g : INT_MIN);
    const double rmax = wave_max(valid ? rn : 0.0);
    const int count = __popcll(__ballot(valid));
    double ctr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ctr[c] = count ? 0.5 * (lo[c] + hi[c]) : 0.0;

    Rec* rec = reinterpret_cast<Rec*>(rec_out);
    if constexpr (MIXED == 0) {
        Rec r;
        r.x = y[0]; r.y = y[1]; r.z = y[2];
        r.qx = q[0]; r.qy = q[1]; r.qz = q[2];
        if constexpr (KT == 1) { r.nx = nv[0]; r.ny = nv[1]; r.nz = nv[2]; r.pad = 0.0; }
        rec[i] = r;
        reinterpret_cast<int32_t*>(aux_out)[i] = g;
    } else {
        // offset from the sub-tile centre as float32 high part + float32 residue
        float hi3[3], lo3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double off = y[c] - ctr[c];
            hi3[c] = valid ? (float)off : kPadOff;
            lo3[c] = valid ? (float)(off - (double)hi3[c]) : 0.0f;
        }
        reinterpret_cast<float4*>(aux_out)[i] = make_float4(lo3[0], lo3[1], lo3[2], 0.0f);
        Rec r;
        r.ox = hi3[0];
        r.oy = hi3[1];
        r.oz = hi3[2];
        r.qx = (float)q[0]; r.qy = (float)q[1]; r.qz = (float)q[2];
        r.t2 = (float)(rn * rn);
        r.g = g;
        if constexpr (KT == 1) { r.nx = (float)nv[0]; r.ny = (float)nv[1]; r.nz = (float)nv[2]; r.pad = 0.f; }
        rec[i] = r;
    }
    if (lane == 0) {
        SubMeta m;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m.lo[c] = count ? lo[c] : 0.0;
            m.hi[c] = count ? hi[c] : 0.0;
            m.ctr[c] = ctr[c];
        }
        m.rnear = rmax;
        m.gmin = gmin; m.gmax = gmax; m.count = count; m.pad = 0;
        meta[i / kSub] = m;
    }
}

// ---------------------------------------------------------------------------
// target setup shared by both precisions
// ---------------------------------------------------------------------------
template <int T>
struct WaveTargets {
    double x[T], y[T], z[T];
    int32_t g[T];
    double lo[3], hi[3];
    int gmin, gmax;
};

template <int T>
__device__ __forceinline__ void load_targets(const SumInputs& in, int64_t tb, int lane,
                                             WaveTargets<T>& t) {
    const int64_t n = in.n_trg;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    int gmn = INT_MAX, gmx = INT_MIN;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t idx = tb + (int64_t)k * kWave + lane;
        const bool v = idx < n;
        const int64_t ic = v ? idx : n - 1;
        t.x[k] = in.trg_xyz[ic];
        t.y[k] = in.trg_xyz[n + ic];
        t.z[k] = in.trg_xyz[2 * n + ic];
        t.g[k] = in.trg_group ? in.trg_group[ic] : 0;
        if (v) {
            lo[0] = fmin(lo[0], t.x[k]); hi[0] = fmax(hi[0], t.x[k]);
            lo[1] = fmin(lo[1], t.y[k]); hi[1] = fmax(hi[1], t.y[k]);
            lo[2] = fmin(lo[2], t.z[k]); hi[2] = fmax(hi[2], t.z[k]);
            gmn = min(gmn, t.g[k]); gmx = max(gmx, t.g[k]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) { t.lo[c] = wave_min(lo[c]); t.hi[c] = wave_max(hi[c]); }
    t.gmin = wave_mini(gmn);
    t.gmax = wave_maxi(gmx);
}

// Squared distance between the wave's target box and a sub-tile box.
template <int T>
__device__ __forceinline__ double box_gap2(const WaveTargets<T>& t, const SubMeta& m) {
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g = fmax(fmax(m.lo[c] - t.hi[c], t.lo[c] - m.hi[c]), 0.0);
        d2 = __builtin_fma(g, g, d2);
    }
    return d2;
}

template <int T>
__device__ __forceinline__ bool groups_overlap(const WaveTargets<T>& t, const SubMeta& m) {
    return !(m.gmax < t.gmin || m.gmin > t.gmax);
}

template <int T>
__device__ __forceinline__ void store_targets(const DirectArgs& a, int64_t tb, int lane,
                                              const double (&ax)[T], const double (&ay)[T],
                                              const double (&az)[T]) {
    const int64_t n = a.in.n_trg;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t idx = tb + (int64_t)k * kWave + lane;
        if (idx >= n) continue;
        if (a.splits == 1) {
            const double p = a.in.pref;
            if (a.accumulate) {
                a.out[idx] += p * ax[k];
                a.out[n + idx] += p * ay[k];
                a.out[2 * n + idx] += p * az[k];
            } else {
                a.out[idx] = p * ax[k];
                a.out[n + idx] = p * ay[k];
                a.out[2 * n + idx] = p * az[k];
            }
        } else {
            double* part = a.out + (int64_t)blockIdx.y * 3 * n;
            part[idx] = ax[k];
            part[n + idx] = ay[k];
            part[2 * n + idx] = az[k];
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 pair kernels (bare, without prefactor)
// ---------------------------------------------------------------------------
template <int KT, bool MASKED>
__device__ __forceinline__ void pair_f64(const typename SrcRec<KT, 0>::type& s, double x, double y,
                                         double z, bool skip, double& ax, double& ay, double& az) {
    const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double ri = MASKED ? rsqrt_nr_masked(r2, skip) : rsqrt_nr(r2);
    const double ri2 = ri * ri;
    const double rq = __builtin_fma(dx, s.qx, __builtin_fma(dy, s.qy, dz * s.qz));
    if constexpr (KT == 0) {
        // q/rho + r (r.q)/rho^3 = (q + r (r.q)/rho^2) / rho
        const double c = rq * ri2;
        ax = __builtin_fma(__builtin_fma(c, dx, s.qx), ri, ax);
        ay = __builtin_fma(__builtin_fma(c, dy, s.qy), ri, ay);
        az = __builtin_fma(__builtin_fma(c, dz, s.qz), ri, az);
    } else {
        // r (r.n)(r.q)/rho^5
        const double rn = __builtin_fma(dx, s.nx, __builtin_fma(dy, s.ny, dz * s.nz));
        const double ri5 = ri2 * ri2 * ri;
        const double c = rn * rq * ri5;
        ax = __builtin_fma(c, dx, ax);
        ay = __builtin_fma(c, dy, ay);
        az = __builtin_fma(c, dz, az);
    }
}

template <int KT, int T>
__global__ __launch_bounds__(kBlock) void direct_f64(DirectArgs a) {
    using Rec = typename SrcRec<KT, 0>::type;
    __shared__ Rec s_rec[kTile];
    __shared__ int32_t s_grp[kTile];

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t tb = (int64_t)blockIdx.x * (kBlock * T) + (int64_t)wave * (kWave * T);
    const bool wave_active = tb < a.in.n_trg;

    WaveTargets<T> t;
    load_targets<T>(a.in, wave_active ? tb : 0, lane, t);
    double ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;

    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    const int64_t sb = (int64_t)blockIdx.y * a.subs_per_split;
    const int64_t se = min(sb + a.subs_per_split, a.n_sub);
    const bool excl = a.in.excl != 0;

    Rec pre;
    int32_t pre_g = 0;
    if (sb < se) {
        pre = rec[sb * kSub + threadIdx.x];
        pre_g = reinterpret_cast<const int32_t*>(a.aux)[sb * kSub + threadIdx.x];
    }
    for (int64_t c = sb; c < se; c += 4) {
        __syncthreads();
        s_rec[threadIdx.x] = pre;
        s_grp[threadIdx.x] = pre_g;
        __syncthreads();
        if (c + 4 < se) {
            pre = rec[(c + 4) * kSub + threadIdx.x];
            pre_g = reinterpret_cast<const int32_t*>(a.aux)[(c + 4) * kSub + threadIdx.x];
        }
        if (!wave_active) continue;
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            const SubMeta m = a.meta[c + s];
            if (m.count == 0) continue;
            const bool slow = (excl && groups_overlap(t, m)) || !(box_gap2(t, m) > 0.0);
            const Rec* base = s_rec + s * kSub;
            if (!slow) {
#pragma unroll 2
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        pair_f64<KT, false>(sr, t.x[k], t.y[k], t.z[k], false, ax[k], ay[k], az[k]);
                }
            } else {
                const int32_t* gb = s_grp + s * kSub;
#pragma unroll 2
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
                    const int32_t gs = gb[j];
#pragma unroll
                    for (int k = 0; k < T; ++k) {
                        const double dx = t.x[k] - sr.x, dy = t.y[k] - sr.y, dz = t.z[k] - sr.z;
                        const bool same = dx == 0.0 && dy == 0.0 && dz == 0.0;
                        const bool skip = same || (excl && gs == t.g[k]);
                        pair_f64<KT, true>(sr, t.x[k], t.y[k], t.z[k], skip, ax[k], ay[k], az[k]);
                    }
                }
            }
        }
    }
    if (wave_active) store_targets<T>(a, tb, lane, ax, ay, az);
}

// ---------------------------------------------------------------------------
// Mixed precision: float32 pairs on centred offsets, float64 near pairs & sums
// ---------------------------------------------------------------------------
template <int KT, bool MASKED>
__device__ __forceinline__ void pair_f32(const typename SrcRec<KT, 1>::type& s, float x, float y,
                                         float z, bool skip, float& ax, float& ay, float& az) {
    const float dx = x - s.ox, dy = y - s.oy, dz = z - s.oz;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float ri = MASKED ? (skip ? 0.0f : __builtin_amdgcn_rsqf(r2)) : __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float rq = __builtin_fmaf(dx, s.qx, __builtin_fmaf(dy, s.qy, dz * s.qz));
    if constexpr (KT == 0) {
        const float c = rq * ri2;
        ax = __builtin_fmaf(__builtin_fmaf(c, dx, s.qx), ri, ax);
        ay = __builtin_fmaf(__builtin_fmaf(c, dy, s.qy), ri, ay);
        az = __builtin_fmaf(__builtin_fmaf(c, dz, s.qz), ri, az);
    } else {
        const float rn = __builtin_fmaf(dx, s.nx, __builtin_fmaf(dy, s.ny, dz * s.nz));
        const float ri5 = ri2 * ri2 * ri;
        const float c = rn * rq * ri5;
        ax = __builtin_fmaf(c, dx, ax);
        ay = __builtin_fmaf(c, dy, ay);
        az = __builtin_fmaf(c, dz, az);
    }
}

// One pair in float64 from the caller's arrays (near pairs of the mixed path).
template <int KT>
__device__ __noinline__ void near_pair_f64(const SumInputs& in, int64_t m, int64_t n_idx,
                                           double& ax, double& ay, double& az) {
    const int64_t ns = in.n_src, nt = in.n_trg;
    const double dx = in.trg_xyz[n_idx] - in.src_xyz[m];
    const double dy = in.trg_xyz[nt + n_idx] - in.src_xyz[ns + m];
    const double dz = in.trg_xyz[2 * nt + n_idx] - in.src_xyz[2 * ns + m];
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

template <int KT, int T>
__global__ __launch_bounds__(kBlock) void direct_mixed(DirectArgs a) {
    using Rec = typename SrcRec<KT, 1>::type;
    __shared__ Rec s_rec[kTile];
    __shared__ float4 s_lo[kTile];

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t tb = (int64_t)blockIdx.x * (kBlock * T) + (int64_t)wave * (kWave * T);
    const bool wave_active = tb < a.in.n_trg;

    WaveTargets<T> t;
    load_targets<T>(a.in, wave_active ? tb : 0, lane, t);
    const double wext = fmax(fmax(t.hi[0] - t.lo[0], t.hi[1] - t.lo[1]), t.hi[2] - t.lo[2]);
    double ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;

    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    const float4* lo = reinterpret_cast<const float4*>(a.aux);
    const int64_t sb = (int64_t)blockIdx.y * a.subs_per_split;
    const int64_t se = min(sb + a.subs_per_split, a.n_sub);
    const bool excl = a.in.excl != 0;

    Rec pre;
    float4 pre_lo;
    if (sb < se) {
        pre = rec[sb * kSub + threadIdx.x];
        pre_lo = lo[sb * kSub + threadIdx.x];
    }
    for (int64_t c = sb; c < se; c += 4) {
        __syncthreads();
        s_rec[threadIdx.x] = pre;
        s_lo[threadIdx.x] = pre_lo;
        __syncthreads();
        if (c + 4 < se) {
            pre = rec[(c + 4) * kSub + threadIdx.x];
            pre_lo = lo[(c + 4) * kSub + threadIdx.x];
        }
        if (!wave_active) continue;
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            const SubMeta m = a.meta[c + s];
            if (m.count == 0) continue;
            // A sub-tile is "close" when it may hold excluded or near pairs, or
            // when its box gap is below half the two boxes' extents: there the
            // float32 offsets' rounding (~eps32 * extent) would be large
            // relative to rho, so r is formed from high + low parts instead.
            const double sext = fmax(fmax(m.hi[0] - m.lo[0], m.hi[1] - m.lo[1]), m.hi[2] - m.lo[2]);
            const double cd0 = fabs(0.5 * (t.lo[0] + t.hi[0]) - m.ctr[0]);
            const double cd1 = fabs(0.5 * (t.lo[1] + t.hi[1]) - m.ctr[1]);
            const double cd2 = fabs(0.5 * (t.lo[2] + t.hi[2]) - m.ctr[2]);
            const double slack = 0x1p-20 * (cd0 + cd1 + cd2 + wext + sext);
            const double lim = fmax(1.001 * m.rnear + slack, 0.5 * (wext + sext));
            const bool close = (excl && groups_overlap(t, m)) || !(box_gap2(t, m) > lim * lim);
            // target offsets from the sub-tile centre, rounded once from float64
            float xs[T], ys[T], zs[T], bx[T], by[T], bz[T];
#pragma unroll
            for (int k = 0; k < T; ++k) {
                xs[k] = (float)(t.x[k] - m.ctr[0]);
                ys[k] = (float)(t.y[k] - m.ctr[1]);
                zs[k] = (float)(t.z[k] - m.ctr[2]);
                bx[k] = by[k] = bz[k] = 0.0f;
            }
            const Rec* base = s_rec + s * kSub;
            if (!close) {
#pragma unroll 2
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        pair_f32<KT, false>(sr, xs[k], ys[k], zs[k], false, bx[k], by[k], bz[k]);
                }
            } else {
                float xl[T], yl[T], zl[T];
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    xl[k] = (float)((t.x[k] - m.ctr[0]) - (double)xs[k]);
                    yl[k] = (float)((t.y[k] - m.ctr[1]) - (double)ys[k]);
                    zl[k] = (float)((t.z[k] - m.ctr[2]) - (double)zs[k]);
                }
                const float4* lb = s_lo + s * kSub;
                const int64_t src0 = (c + s) * kSub;
#pragma unroll 1
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
                    const float4 sl = lb[j];
#pragma unroll
                    for (int k = 0; k < T; ++k) {
                        // r = (x_hi - y_hi) + (x_lo - y_lo): the high difference is
                        // rounded relative to rho, the residues carry the rest
                        const float dx = (xs[k] - sr.ox) + (xl[k] - sl.x);
                        const float dy = (ys[k] - sr.oy) + (yl[k] - sl.y);
                        const float dz = (zs[k] - sr.oz) + (zl[k] - sl.z);
                        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                        const bool excluded = excl && sr.g == t.g[k];
                        const bool near = r2 <= sr.t2;
                        const bool skip = excluded || near;
                        const float ri = skip ? 0.0f : __builtin_amdgcn_rsqf(r2);
                        const float ri2 = ri * ri;
                        const float rq = __builtin_fmaf(dx, sr.qx, __builtin_fmaf(dy, sr.qy, dz * sr.qz));
                        if constexpr (KT == 0) {
                            const float cc = rq * ri2;
                            bx[k] = __builtin_fmaf(__builtin_fmaf(cc, dx, sr.qx), ri, bx[k]);
                            by[k] = __builtin_fmaf(__builtin_fmaf(cc, dy, sr.qy), ri, by[k]);
                            bz[k] = __builtin_fmaf(__builtin_fmaf(cc, dz, sr.qz), ri, bz[k]);
                        } else {
                            const float rn = __builtin_fmaf(dx, sr.nx, __builtin_fmaf(dy, sr.ny, dz * sr.nz));
                            const float cc = rn * rq * (ri2 * ri2 * ri);
                            bx[k] = __builtin_fmaf(cc, dx, bx[k]);
                            by[k] = __builtin_fmaf(cc, dy, by[k]);
                            bz[k] = __builtin_fmaf(cc, dz, bz[k]);
                        }
                        if (near && !excluded) {
                            const int64_t idx = tb + (int64_t)k * kWave + lane;
                            const int64_t ic = idx < a.in.n_trg ? idx : a.in.n_trg - 1;
                            near_pair_f64<KT>(a.in, src0 + j, ic, ax[k], ay[k], az[k]);
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < T; ++k) {
                ax[k] += (double)bx[k];
                ay[k] += (double)by[k];
                az[k] += (double)bz[k];
            }
        }
    }
    if (wave_active) store_targets<T>(a, tb, lane, ax, ay, az);
}

// ---------------------------------------------------------------------------
// split reduction and fills
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void reduce_splits(const double* __restrict__ part, int splits,
                                                        int64_t n3, double pref, double* out,
                                                        int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n3) return;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += part[(int64_t)k * n3 + i];
    out[i] = accumulate ? out[i] + pref * s : pref * s;
}

__global__ __launch_bounds__(kBlock) void fill_zero(double* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = 0.0;
}

hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    fill_zero<<<dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, stream>>>(out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// planning and launch
// ---------------------------------------------------------------------------
static int targets_per_lane(int kernel, int mixed) {
    (void)kernel;
    (void)mixed;
    return 4;
}

static size_t rec_bytes(int kernel, int mixed) {
    if (!mixed) return kernel == 0 ? sizeof(SrcSL64) : sizeof(SrcDL64);
    return kernel == 0 ? sizeof(SrcSL32) : sizeof(SrcDL32);
}

DirectPlan plan_direct(int kernel, int mixed, int64_t n_src, int64_t n_trg, int n_cu,
                       int forced_splits) {
    DirectPlan p{};
    p.T = targets_per_lane(kernel, mixed);
    p.n_src_pad = ceil_div(n_src, kTile) * kTile;
    p.n_sub = p.n_src_pad / kSub;
    p.blocks_x = ceil_div(n_trg, (int64_t)kBlock * p.T);
    const int64_t chunks = p.n_sub / 4;
    int64_t splits = 1;
    if (chunks > 0 && p.blocks_x > 0) {
        if (forced_splits > 0) {
            splits = forced_splits;
        } else {
            // aim for ~4 waves per SIMD (16 per CU) while keeping >= 2 chunks per split
            const int64_t want_waves = (int64_t)n_cu * 16;
            const int64_t waves = p.blocks_x * 4;
            splits = ceil_div(want_waves, waves);
            splits = std::min<int64_t>(splits, std::max<int64_t>(1, chunks / 2));
        }
        splits = std::max<int64_t>(1, std::min<int64_t>(splits, chunks));
    }
    int64_t per = chunks > 0 ? ceil_div(chunks, splits) : 0;
    if (per > 0) splits = ceil_div(chunks, per);   // drop empty splits
    p.splits = (int)splits;
    p.subs_per_split = per * 4;
    size_t off = 0;
    p.off_src = off;
    off = align_up(off + (size_t)p.n_src_pad * rec_bytes(kernel, mixed), 256);
    p.off_grp = off;
    off = align_up(off + (size_t)p.n_src_pad * (mixed ? sizeof(float4) : sizeof(int32_t)), 256);
    p.off_meta = off;
    off = align_up(off + (size_t)p.n_sub * sizeof(SubMeta), 256);
    p.off_part = off;
    if (p.splits > 1) off = align_up(off + (size_t)p.splits * 3 * (size_t)n_trg * sizeof(double), 256);
    p.total = off;
    return p;
}

template <int KT, int MIXED>
static hipError_t launch_typed(const SumInputs& in, const DirectPlan& p, double* out, int accumulate,
                               void* ws, hipStream_t stream) {
    char* base = static_cast<char*>(ws);
    void* rec = base + p.off_src;
    void* aux = base + p.off_grp;
    SubMeta* meta = reinterpret_cast<SubMeta*>(base + p.off_meta);
    prep_sources<KT, MIXED><<<dim3((unsigned)(p.n_src_pad / kBlock)), dim3(kBlock), 0, stream>>>(
        in, rec, aux, meta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    DirectArgs a;
    a.in = in;
    a.rec = rec;
    a.aux = aux;
    a.meta = meta;
    a.n_sub = p.n_sub;
    a.subs_per_split = p.subs_per_split;
    a.splits = p.splits;
    a.accumulate = accumulate;
    a.out = p.splits > 1 ? reinterpret_cast<double*>(base + p.off_part) : out;
    const dim3 grid((unsigned)p.blocks_x, (unsigned)p.splits);
    if (MIXED) {
        direct_mixed<KT, 4><<<grid, dim3(kBlock), 0, stream>>>(a);
    } else {
        direct_f64<KT, 4><<<grid, dim3(kBlock), 0, stream>>>(a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p.splits > 1) {
        const int64_t n3 = 3 * in.n_trg;
        reduce_splits<<<dim3((unsigned)ceil_div(n3, kBlock)), dim3(kBlock), 0, stream>>>(
            reinterpret_cast<const double*>(base + p.off_part), p.splits, n3, in.pref, out, accumulate);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_direct(const SumInputs& in, const DirectPlan& p, double* out, int accumulate,
                         void* ws, hipStream_t stream) {
    if (in.n_trg <= 0) return hipSuccess;
    if (in.n_src <= 0) return accumulate ? hipSuccess : launch_fill_zero(out, 3 * in.n_trg, stream);
    if (in.kernel == 0) {
        return in.mixed ? launch_typed<0, 1>(in, p, out, accumulate, ws, stream)
                        : launch_typed<0, 0>(in, p, out, accumulate, ws, stream);
    }
    return in.mixed ? launch_typed<1, 1>(in, p, out, accumulate, ws, stream)
                    : launch_typed<1, 0>(in, p, out, accumulate, ws, stream);
}

}  // namespace stokes
