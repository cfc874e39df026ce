// Direct (all-pairs) Stokes kernel sums on gfx950.
//
// Single layer (Stokeslet, paper eq. sl_stokes) and double layer (stresslet,
// stated after eq. double_layer_int_eq), summed over the smooth quadrature of
// eq. smooth_double_layer_int_eq_patches_disc (strength q = w * density),
// with the "other cells only" rule of the explicit step (Sec. 2.2, step 1(d))
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
//   * per 64-source sub-tile the wave decides, uniformly, whether the fast
//     loop (no per-pair tests) is exact: box far from its targets and no
//     shared group.  Sub-tiles that need per-pair tests are flagged and left
//     to a separate near-pass kernel, so the main loop's register allocation
//     and schedule carry no masked code.  Mixed precision evaluates pairs in float32
//     on offsets from the sub-tile centre (each rounded once from float64),
//     sums each sub-tile in float32 and adds it into float64 accumulators.
//     In the near pass (possible exclusions or near pairs, or a gap below half
//     the sub-tile's extent) r is formed from float32 high parts plus float32
//     residues, and pairs within the near radius are evaluated in float64.
//   * work balance (stream-K): the grid holds exactly the resident number of
//     workgroups; the (target block x source chunk) units are cut into equal
//     contiguous ranges, one per workgroup.  A workgroup flushes float64
//     partial sums whenever its range moves to a new target block; segment
//     ids (workgroup + target block) are consecutive, and a second kernel
//     adds each target's segments in fixed order (deterministic, no atomics).
//   * the near-pass decision tests every target of the wave against the
//     sub-tile box, after a whole-wave box test that settles most sub-tiles.
#include <float.h>
#include <limits.h>

#include "direct_dev.hpp"

namespace stokes {

struct DirectArgs {
    SumInputs in;
    const void* rec;          // packed source records
    const void* aux;          // FP64 path: padded int32 groups; mixed: float4 low parts
    const SubMeta* meta;
    int64_t chunks;           // source chunks of kTile records
    int64_t units;            // target blocks x chunks
    double* part;             // partial sums, one segment per (block, target block) pair
    uint8_t* flags;           // per (wave, chunk): bit s = sub-tile s left to the near pass
    double* near_part;        // near-pass sums, (kNearSlices, 3, blocks_x * kBlock * T)
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
        if (MIXED == 0) {   // FP64 records hold doubled positions (exact)
            y[0] *= 2.0; y[1] *= 2.0; y[2] *= 2.0;
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
        if constexpr (KT == 0) { r.q4x = 4.0 * q[0]; r.q4y = 4.0 * q[1]; r.q4z = 4.0 * q[2]; r.pad = 0.0; }
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

template <int T>
__device__ __forceinline__ void flush_segment(const DirectArgs& a, int64_t tbk, int wave, int lane,
                                              const double (&ax)[T], const double (&ay)[T],
                                              const double (&az)[T]) {
    constexpr int BT = kBlock * T;
    double* seg = a.part + (int64_t)(blockIdx.x + tbk) * 3 * BT;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int li = wave * (kWave * T) + k * kWave + lane;
        seg[li] = ax[k];
        seg[BT + li] = ay[k];
        seg[2 * BT + li] = az[k];
    }
}

// Launch-shape tuning: targets per lane (T) and the minimum number of waves
// per SIMD that the register allocation must allow, for each precision.
#ifndef STOKES_DIRECT_T64
#define STOKES_DIRECT_T64 4
#endif
#ifndef STOKES_DIRECT_W64
#define STOKES_DIRECT_W64 3
#endif
#ifndef STOKES_DIRECT_T32
#define STOKES_DIRECT_T32 2
#endif
#ifndef STOKES_DIRECT_W32
#define STOKES_DIRECT_W32 4
#endif

// Main FP64 kernel: fast loop only; sub-tiles needing per-pair tests are
// flagged for direct_near_f64.
template <int KT, int T>
__global__ __launch_bounds__(kBlock, STOKES_DIRECT_W64) void direct_f64(DirectArgs a) {
    using Rec = typename SrcRec<KT, 0>::type;
    constexpr int BT = kBlock * T;
    __shared__ Rec s_rec[kTile];

    const int64_t U = a.units, C = a.chunks, G = gridDim.x;
    const int64_t u0 = unit_begin(blockIdx.x, U, G), u1 = unit_begin(blockIdx.x + 1, U, G);
    if (u0 >= u1) return;                      // whole workgroup idle (uniform)
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const bool excl = a.in.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);

    Targets<T> t;
    Box wbox{};
    bool wave_active = false;
    int64_t tbk = -1;
    double ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;

    int64_t ub = u0 / C, c = u0 % C;           // unit position, advanced incrementally
    for (int64_t u = u0; u < u1; ++u) {
        __syncthreads();                       // previous step's readers are done
        if (ub != tbk) {
            if (tbk >= 0) flush_segment<T>(a, tbk, wave, lane, ax, ay, az);
            tbk = ub;
            const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
            wave_active = tb < a.in.n_trg;
            wbox = load_targets<T>(a.in, wave_active ? tb : 0, lane, t);
            double_targets<T>(t, &wbox);
#pragma unroll
            for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;
        }
        s_rec[threadIdx.x] = rec[c * kTile + threadIdx.x];
        __syncthreads();
        int64_t cn = c + 1, ubn = ub;
        if (cn == C) { cn = 0; ++ubn; }
        if (wave_active) {
            uint32_t flags = 0;
#pragma unroll 1
            for (int s = 0; s < 4; ++s) {
                const SubMeta m = a.meta[c * 4 + s];
                if (m.count == 0) continue;
                if (needs_near<T, false>(wbox, t, m, excl)) {
                    flags |= 1u << s;
                    continue;
                }
                const Rec* base = s_rec + s * kSub;
#pragma unroll 2
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        pair_f64<KT, false>(sr, t.x[k], t.y[k], t.z[k], false, ax[k], ay[k], az[k]);
                }
            }
            if (lane == 0) a.flags[(tbk * 4 + wave) * C + c] = (uint8_t)flags;
        }
        c = cn;
        ub = ubn;
    }
    flush_segment<T>(a, tbk, wave, lane, ax, ay, az);
}

// Near pass (FP64): for each wave of each target block, the flagged
// sub-tiles with the same-group and zero-distance masks.
template <int KT, int T>
__global__ __launch_bounds__(kBlock) void direct_near_f64(DirectArgs a) {
    using Rec = typename SrcRec<KT, 0>::type;
    constexpr int BT = kBlock * T;
    // per-wave staging slice of the current sub-tile (see direct_near_mixed)
    __shared__ Rec s_src[4][kSub];
    __shared__ int32_t s_grp[4][kSub];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t tbk = blockIdx.x, C = a.chunks;
    const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
    if (tb >= a.in.n_trg) return;              // wave has no targets (no barriers below)
    const bool excl = a.in.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    const int32_t* grp = reinterpret_cast<const int32_t*>(a.aux);
    Targets<T> t;
    (void)load_targets<T>(a.in, tb, lane, t);
    double_targets<T>(t, nullptr);
    double ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;
    const uint8_t* fl = a.flags + (tbk * 4 + wave) * C;
    for_each_flagged(fl, C, lane, (int)blockIdx.y, [&](int64_t sub) {
        s_src[wave][lane] = rec[sub * kSub + lane];
        s_grp[wave][lane] = grp[sub * kSub + lane];
        __builtin_amdgcn_wave_barrier();
#pragma unroll 2
        for (int j = 0; j < kSub; ++j) {
            const Rec sr = s_src[wave][j];
            const int32_t gs = s_grp[wave][j];
#pragma unroll
            for (int k = 0; k < T; ++k)
                pair_f64<KT, true>(sr, t.x[k], t.y[k], t.z[k], excl && gs == t.g[k], ax[k], ay[k],
                                   az[k]);
        }
        __builtin_amdgcn_wave_barrier();   // reads of this sub-tile precede the next writes
    });
    const int64_t np = (int64_t)gridDim.x * BT;
    double* np_slice = a.near_part + (int64_t)blockIdx.y * 3 * np;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t gi = tbk * BT + wave * (kWave * T) + k * kWave + lane;
        np_slice[gi] = ax[k];
        np_slice[np + gi] = ay[k];
        np_slice[2 * np + gi] = az[k];
    }
}

// Main mixed kernel: float32 fast loop only; sub-tiles needing care are
// flagged for direct_near_mixed.  CNT: also record each pair's class
// (test-only instantiation).
template <int KT, int T, bool CNT = false>
__global__ __launch_bounds__(kBlock, STOKES_DIRECT_W32) void direct_mixed(DirectArgs a) {
    using Rec = typename SrcRec<KT, 1>::type;
    constexpr int BT = kBlock * T;
    __shared__ Rec s_rec[kTile];

    const int64_t U = a.units, C = a.chunks, G = gridDim.x;
    const int64_t u0 = unit_begin(blockIdx.x, U, G), u1 = unit_begin(blockIdx.x + 1, U, G);
    if (u0 >= u1) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const bool excl = a.in.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);

    Targets<T> t;
    Box wbox{};
    bool wave_active = false;
    int64_t tbk = -1;
    double ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;

    int64_t ub = u0 / C, c = u0 % C;
    Rec pre = rec[c * kTile + threadIdx.x];
    for (int64_t u = u0; u < u1; ++u) {
        __syncthreads();
        if (ub != tbk) {
            if (tbk >= 0) flush_segment<T>(a, tbk, wave, lane, ax, ay, az);
            tbk = ub;
            const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
            wave_active = tb < a.in.n_trg;
            wbox = load_targets<T>(a.in, wave_active ? tb : 0, lane, t);
#pragma unroll
            for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;
        }
        s_rec[threadIdx.x] = pre;
        __syncthreads();
        int64_t cn = c + 1, ubn = ub;
        if (cn == C) { cn = 0; ++ubn; }
        if (u + 1 < u1) pre = rec[cn * kTile + threadIdx.x];
        if (wave_active) {
            uint32_t flags = 0;
#pragma unroll 1
            for (int s = 0; s < 4; ++s) {
                const SubMeta m = a.meta[c * 4 + s];
                if (m.count == 0) continue;
                if (needs_near<T, true>(wbox, t, m, excl)) {
                    flags |= 1u << s;
                    continue;
                }
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
#pragma unroll 2
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        pair_f32<KT>(sr, xs[k] - sr.ox, ys[k] - sr.oy, zs[k] - sr.oz, false, false,
                                     bx[k], by[k], bz[k]);
                }
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    ax[k] += (double)bx[k];
                    ay[k] += (double)by[k];
                    az[k] += (double)bz[k];
                }
                if constexpr (CNT) {
                    const int64_t s0 = c * kTile + s * kSub;
                    for (int k = 0; k < T; ++k) {
                        const int64_t ti = tbk * BT + (int64_t)wave * (kWave * T) + k * kWave + lane;
                        if (ti < a.in.n_trg)
                            for (int j = 0; j < m.count; ++j)
                                atomicAdd(a.in.pair_class + ti * a.in.n_src + s0 + j, kPairF32);
                    }
                }
            }
            if (lane == 0) a.flags[(tbk * 4 + wave) * C + c] = (uint8_t)flags;
        }
        c = cn;
        ub = ubn;
    }
    flush_segment<T>(a, tbk, wave, lane, ax, ay, az);
}

// Near pass (mixed): flagged sub-tiles with r from high + low float32 parts,
// the same-group mask, and pairs inside the near radius in float64.  CNT:
// also record each pair's class (test-only instantiation).
template <int KT, int T, bool CNT = false>
__global__ __launch_bounds__(kBlock) void direct_near_mixed(DirectArgs a) {
    using Rec = typename SrcRec<KT, 1>::type;
    constexpr int BT = kBlock * T;
    // each wave stages its current sub-tile in its own slice (read back by
    // broadcast into VGPRs; only that wave touches it, and a wave's LDS
    // operations complete in order, so no workgroup barrier is needed)
    __shared__ Rec s_src[4][kSub];
    __shared__ float4 s_res[4][kSub];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t tbk = blockIdx.x, C = a.chunks;
    const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
    if (tb >= a.in.n_trg) return;
    const bool excl = a.in.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    const float4* lo = reinterpret_cast<const float4*>(a.aux);
    Targets<T> t;
    (void)load_targets<T>(a.in, tb, lane, t);
    double ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;
    const uint8_t* fl = a.flags + (tbk * 4 + wave) * C;
    for_each_flagged(fl, C, lane, (int)blockIdx.y, [&](int64_t sub) {
        const SubMeta m = a.meta[sub];
        float xs[T], ys[T], zs[T], xl[T], yl[T], zl[T], bx[T], by[T], bz[T];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const double hx = t.x[k] - m.ctr[0], hy = t.y[k] - m.ctr[1], hz = t.z[k] - m.ctr[2];
            xs[k] = (float)hx; ys[k] = (float)hy; zs[k] = (float)hz;
            xl[k] = (float)(hx - (double)xs[k]);
            yl[k] = (float)(hy - (double)ys[k]);
            zl[k] = (float)(hz - (double)zs[k]);
            bx[k] = by[k] = bz[k] = 0.0f;
        }
        s_src[wave][lane] = rec[sub * kSub + lane];
        s_res[wave][lane] = lo[sub * kSub + lane];
        __builtin_amdgcn_wave_barrier();
#pragma unroll 2
        for (int j = 0; j < kSub; ++j) {
            const Rec sr = s_src[wave][j];
            const float4 sl = s_res[wave][j];
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
                pair_f32<KT>(sr, dx, dy, dz, excluded || near, true, bx[k], by[k], bz[k]);
                if (near && !excluded)
                    near_pair_f64<KT>(a.in, sub * kSub + j, t.x[k], t.y[k], t.z[k], ax[k], ay[k],
                                      az[k]);
                if constexpr (CNT) {
                    const int64_t si = sub * kSub + j, ti = tb + k * kWave + lane;
                    if (si < a.in.n_src && ti < a.in.n_trg) {
                        // near_pair_f64 takes nothing at zero distance (float64)
                        const int64_t ns = a.in.n_src;
                        const bool zero = t.x[k] == a.in.src_xyz[si] && t.y[k] == a.in.src_xyz[ns + si] &&
                                          t.z[k] == a.in.src_xyz[2 * ns + si];
                        const int32_t cls = excluded ? kPairSkip : !near ? kPairF32 : zero ? kPairSkip : kPairF64;
                        atomicAdd(a.in.pair_class + ti * ns + si, cls);
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
        __builtin_amdgcn_wave_barrier();   // reads of this sub-tile precede the next writes
    });
    const int64_t np = (int64_t)gridDim.x * BT;
    double* np_slice = a.near_part + (int64_t)blockIdx.y * 3 * np;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t gi = tbk * BT + wave * (kWave * T) + k * kWave + lane;
        np_slice[gi] = ax[k];
        np_slice[np + gi] = ay[k];
        np_slice[2 * np + gi] = az[k];
    }
}

// ---------------------------------------------------------------------------
// segment reduction and fills
// ---------------------------------------------------------------------------
// out[c][i] (=|+=) pref * (sum of target i's segments in workgroup order
//                          + its near-pass sum).
template <int T>
__global__ __launch_bounds__(kBlock) void reduce_segments(const double* __restrict__ part,
                                                          const double* __restrict__ near_part,
                                                          int64_t n_trg, int64_t units,
                                                          int64_t chunks, int64_t grid,
                                                          int64_t np, double pref, double* out,
                                                          int accumulate) {
    constexpr int BT = kBlock * T;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_trg) return;
    const int64_t tbk = i / BT, li = i % BT;
    const int64_t b0 = unit_owner(tbk * chunks, units, grid);
    const int64_t b1 = unit_owner((tbk + 1) * chunks - 1, units, grid);
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t b = b0; b <= b1; ++b) {
        const double* seg = part + (b + tbk) * 3 * BT;
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += seg[c * BT + li];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        for (int sl = 0; sl < kNearSlices; ++sl) s[c] += near_part[(sl * 3 + c) * np + i];
        const int64_t o = c * n_trg + i;
        out[o] = accumulate ? out[o] + pref * s[c] : pref * s[c];
    }
}

hipError_t launch_prep(const SumInputs& in, int64_t n_pad, void* rec, void* aux, SubMeta* meta,
                       hipStream_t stream) {
    const dim3 grid((unsigned)(n_pad / kBlock)), block(kBlock);
    if (in.kernel == 0) {
        if (in.mixed) prep_sources<0, 1><<<grid, block, 0, stream>>>(in, rec, aux, meta);
        else prep_sources<0, 0><<<grid, block, 0, stream>>>(in, rec, aux, meta);
    } else {
        if (in.mixed) prep_sources<1, 1><<<grid, block, 0, stream>>>(in, rec, aux, meta);
        else prep_sources<1, 0><<<grid, block, 0, stream>>>(in, rec, aux, meta);
    }
    return hipGetLastError();
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
constexpr int kT64 = STOKES_DIRECT_T64;
constexpr int kT32 = STOKES_DIRECT_T32;

static size_t rec_bytes(int kernel, int mixed) {
    if (!mixed) return kernel == 0 ? sizeof(SrcSL64x) : sizeof(SrcDL64);
    return kernel == 0 ? sizeof(SrcSL32) : sizeof(SrcDL32);
}

int direct_blocks_per_cu(int kernel, int mixed) {
    int nb = 0;
    hipError_t e;
    if (kernel == 0)
        e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, direct_mixed<0, kT32>, kBlock, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, direct_f64<0, kT64>, kBlock, 0);
    else
        e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, direct_mixed<1, kT32>, kBlock, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, direct_f64<1, kT64>, kBlock, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

DirectPlan plan_direct(int kernel, int mixed, int64_t n_src, int64_t n_trg, int resident_blocks,
                       int forced_grid) {
    DirectPlan p{};
    p.T = mixed ? kT32 : kT64;
    p.n_src_pad = ceil_div(n_src, kTile) * kTile;
    p.n_sub = p.n_src_pad / kSub;
    p.chunks = p.n_src_pad / kTile;
    p.blocks_x = ceil_div(n_trg, (int64_t)kBlock * p.T);
    p.units = p.chunks * p.blocks_x;
    const int64_t g = forced_grid > 0 ? forced_grid : std::max(1, resident_blocks);
    p.grid = std::max<int64_t>(1, std::min<int64_t>(g, p.units));
    const size_t bt = (size_t)kBlock * p.T;
    size_t off = 0;
    p.off_src = off;
    off = align_up(off + (size_t)p.n_src_pad * rec_bytes(kernel, mixed), 256);
    p.off_grp = off;
    off = align_up(off + (size_t)p.n_src_pad * (mixed ? sizeof(float4) : sizeof(int32_t)), 256);
    p.off_meta = off;
    off = align_up(off + (size_t)p.n_sub * sizeof(SubMeta), 256);
    p.off_part = off;
    off = align_up(off + (size_t)(p.grid + p.blocks_x) * 3 * bt * sizeof(double), 256);
    p.off_near = off;
    off = align_up(off + (size_t)kNearSlices * p.blocks_x * 3 * bt * sizeof(double), 256);
    p.off_flags = off;
    off = align_up(off + (size_t)p.blocks_x * 4 * (size_t)p.chunks, 256);
    p.total = off;
    return p;
}

template <int KT, int MIXED>
static hipError_t launch_typed(const SumInputs& in, const DirectPlan& p, double* out, int accumulate,
                               void* ws, hipStream_t stream, const KernelTimer& timer) {
    constexpr int T = MIXED ? kT32 : kT64;
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
    a.chunks = p.chunks;
    a.units = p.units;
    a.part = reinterpret_cast<double*>(base + p.off_part);
    a.near_part = reinterpret_cast<double*>(base + p.off_near);
    a.flags = reinterpret_cast<uint8_t*>(base + p.off_flags);
    if (timer.on()) (void)hipEventRecord(timer.start, stream);
    if constexpr (MIXED != 0) {
        if (in.pair_class)
            direct_mixed<KT, T, true><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
        else
            direct_mixed<KT, T><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
    } else
        direct_f64<KT, T><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (timer.on()) (void)hipEventRecord(timer.stop, stream);
    if (e != hipSuccess) return e;
    if constexpr (MIXED != 0) {
        if (in.pair_class)
            direct_near_mixed<KT, T, true><<<dim3((unsigned)p.blocks_x, kNearSlices), dim3(kBlock), 0, stream>>>(a);
        else
            direct_near_mixed<KT, T><<<dim3((unsigned)p.blocks_x, kNearSlices), dim3(kBlock), 0, stream>>>(a);
    } else
        direct_near_f64<KT, T><<<dim3((unsigned)p.blocks_x, kNearSlices), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // FP64 pair sums are 4x (single layer) or 8x (double layer) the bare sums
    const double pref = MIXED ? in.pref : (KT == 0 ? 0.25 : 0.125) * in.pref;
    reduce_segments<T><<<dim3((unsigned)ceil_div(in.n_trg, kBlock)), dim3(kBlock), 0, stream>>>(
        a.part, a.near_part, in.n_trg, p.units, p.chunks, p.grid, p.blocks_x * (int64_t)kBlock * T,
        pref, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_direct(const SumInputs& in, const DirectPlan& p, double* out, int accumulate,
                         void* ws, hipStream_t stream, const KernelTimer& timer) {
    if (in.n_trg <= 0) return hipSuccess;
    if (in.n_src <= 0) return accumulate ? hipSuccess : launch_fill_zero(out, 3 * in.n_trg, stream);
    if (in.kernel == 0) {
        return in.mixed ? launch_typed<0, 1>(in, p, out, accumulate, ws, stream, timer)
                        : launch_typed<0, 0>(in, p, out, accumulate, ws, stream, timer);
    }
    return in.mixed ? launch_typed<1, 1>(in, p, out, accumulate, ws, stream, timer)
                    : launch_typed<1, 0>(in, p, out, accumulate, ws, stream, timer);
}

}  // namespace stokes
