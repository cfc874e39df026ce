// Generic float64 pair-sum skeleton for gfx950, shared by the adjoint sums.
//
// A pass sums, for every target, a pair function over all sources (minus the
// same-group and zero-distance pairs), into NACC float64 accumulators.  The
// layout and scheduling are those of the direct sums:
//   * prep: one thread per source builds a packed record (policy-defined) and
//     each wave summarises its 64-source sub-tile (box, group range);
//   * main: stream-K split of (target block x 256-source chunk) units over
//     the resident workgroups; sources staged through LDS and read by
//     broadcast; per sub-tile a uniform test (a target of the wave inside the
//     sub-tile box, or a shared group id) sends it to the near pass, every
//     other sub-tile runs the unmasked loop;
//   * near: the flagged sub-tiles with per-pair masks (each wave stages its
//     sub-tile in LDS), in kNearSlices grid rows;
//   * reduce: fixed-order sum of segments and near partials, then the
//     policy's store (scaling, accumulate, output mapping).
//
// A policy P provides:
//   using Rec;                            packed source record (16-byte aligned)
//   static constexpr int NACC, NT;        accumulators per target, extra per-target doubles
//   static void make_rec(const PassArgs&, int64_t i, Rec&, double pos[3]);   prep
//   static void pad_rec(Rec&);            record of a padding source (zero strength, far away)
//   static void load_t(const PassArgs&, int64_t i, double (&tv)[NT]);        per-target data
//   template <bool MASKED> static void pair(const Rec&, double x, double y, double z,
//                                           const double (&tv)[NT], bool skip, double (&acc)[NACC]);
//   static void store(const PassArgs&, int64_t i, const double (&s)[NACC]);
#pragma once

#include <float.h>
#include <limits.h>

#include "common.hpp"

namespace stokes {
namespace ps {

// Arguments of one pass; the policy gives the array fields their meaning.
struct PassArgs {
    // targets of the pass
    int64_t n_trg;
    const double* trg_xyz;      // (3, n_trg)
    const int32_t* trg_group;   // (n_trg) or null
    const double* tv[3];        // per-target arrays
    // sources of the pass (prep inputs)
    int64_t n_src;
    const double* src_xyz;      // (3, n_src)
    const double* sv[3];        // per-source arrays
    const int32_t* src_group;   // (n_src) or null
    int excl;
    // workspace
    void* rec;
    int32_t* grp;
    SubMeta* meta;
    int64_t chunks, units;
    double* part;
    double* near_part;
    uint8_t* flags;
    // outputs
    double* out[3];
    double pref;
    int accumulate;
    const double* force_acc;    // this output adds into its array whatever `accumulate` says
};

__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wmini(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wmaxi(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// 1/sqrt(r2): hardware estimate (~24 bits) + one Newton step; 0 when skip.
__device__ __forceinline__ double rinv(double r2) {
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    return __builtin_fma(0.5 * y0, e, y0);
}
__device__ __forceinline__ double rinv_masked(double r2, bool skip) {
    const double y0 = skip ? 0.0 : __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    return __builtin_fma(0.5 * y0, e, y0);
}

// The near pass takes each wave's flagged sub-tiles in kNearSlices
// interleaved slices (one per grid row, for balance), each writing its own
// partials; the reduction adds the slices in a fixed order.
constexpr int kNearSlices = 4;

// Visits the flagged sub-tiles of one wave's flag row that fall in `slice`.
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
template <class P>
__global__ __launch_bounds__(kBlock) void prep(PassArgs a) {
    using Rec = typename P::Rec;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;   // grid covers the padding
    const int lane = threadIdx.x & (kWave - 1);
    const bool valid = i < a.n_src;
    Rec r;
    double pos[3] = {0.0, 0.0, 0.0};
    int32_t g = INT_MIN;
    if (valid) {
        P::make_rec(a, i, r, pos);
        g = a.src_group ? a.src_group[i] : 0;
    } else {
        P::pad_rec(r);
    }
    reinterpret_cast<Rec*>(a.rec)[i] = r;
    a.grp[i] = g;
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = wmin(valid ? pos[c] : DBL_MAX);
        hi[c] = wmax(valid ? pos[c] : -DBL_MAX);
    }
    const int gmin = wmini(valid ? g : INT_MAX);
    const int gmax = wmaxi(valid ? g : INT_MIN);
    const int count = __popcll(__ballot(valid));
    if (lane == 0) {
        SubMeta m;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            m.lo[c] = count ? lo[c] : 0.0;
            m.hi[c] = count ? hi[c] : 0.0;
            m.ctr[c] = count ? 0.5 * (lo[c] + hi[c]) : 0.0;
        }
        m.rnear = 0.0;
        m.gmin = gmin; m.gmax = gmax; m.count = count; m.pad = 0;
        a.meta[i / kSub] = m;
    }
}

template <class P, int T>
struct Tgt {
    double x[T], y[T], z[T];
    double v[T][P::NT > 0 ? P::NT : 1];
    int32_t g[T];
    double lo[3], hi[3];
    int gmin, gmax;
};

template <class P, int T>
__device__ __forceinline__ void load_tgt(const PassArgs& a, int64_t tb, int lane, Tgt<P, T>& t) {
    const int64_t n = a.n_trg;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    int gmn = INT_MAX, gmx = INT_MIN;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t idx = tb + (int64_t)k * kWave + lane;
        const int64_t ic = idx < n ? idx : n - 1;
        t.x[k] = a.trg_xyz[ic];
        t.y[k] = a.trg_xyz[n + ic];
        t.z[k] = a.trg_xyz[2 * n + ic];
        t.g[k] = a.trg_group ? a.trg_group[ic] : 0;
        if constexpr (P::NT > 0) P::load_t(a, ic, t.v[k]);
        lo[0] = fmin(lo[0], t.x[k]); hi[0] = fmax(hi[0], t.x[k]);
        lo[1] = fmin(lo[1], t.y[k]); hi[1] = fmax(hi[1], t.y[k]);
        lo[2] = fmin(lo[2], t.z[k]); hi[2] = fmax(hi[2], t.z[k]);
        gmn = min(gmn, t.g[k]);
        gmx = max(gmx, t.g[k]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) { t.lo[c] = wmin(lo[c]); t.hi[c] = wmax(hi[c]); }
    t.gmin = wmini(gmn);
    t.gmax = wmaxi(gmx);
}

// Uniform: does any target of the wave touch the sub-tile box, or share a
// group id in its range (same-group rule on)?
template <class P, int T>
__device__ __forceinline__ bool needs_near(const Tgt<P, T>& t, const SubMeta& m, bool excl) {
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g = fmax(fmax(m.lo[c] - t.hi[c], t.lo[c] - m.hi[c]), 0.0);
        d2 = __builtin_fma(g, g, d2);
    }
    const bool gov = !(m.gmax < t.gmin || m.gmin > t.gmax);
    if (!((excl && gov) || !(d2 > 1e-200))) return false;
    bool any = false;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const double p[3] = {t.x[k], t.y[k], t.z[k]};
        double e2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double g = fmax(fmax(m.lo[c] - p[c], p[c] - m.hi[c]), 0.0);
            e2 = __builtin_fma(g, g, e2);
        }
        any |= (excl && t.g[k] >= m.gmin && t.g[k] <= m.gmax) || !(e2 > 1e-200);
    }
    return __ballot(any) != 0;
}

__device__ __forceinline__ int64_t unit_begin(int64_t b, int64_t U, int64_t G) { return b * U / G; }
__device__ __forceinline__ int64_t unit_owner(int64_t u, int64_t U, int64_t G) {
    return ((u + 1) * G - 1) / U;
}

template <class P, int T>
__device__ __forceinline__ void flush(const PassArgs& a, int64_t tbk, int wave, int lane,
                                      const double (&acc)[T][P::NACC]) {
    constexpr int BT = kBlock * T;
    double* seg = a.part + (int64_t)(blockIdx.x + tbk) * P::NACC * BT;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int li = wave * (kWave * T) + k * kWave + lane;
#pragma unroll
        for (int c = 0; c < P::NACC; ++c) seg[c * BT + li] = acc[k][c];
    }
}

template <class P, int T, int W>
__global__ __launch_bounds__(kBlock, W) void main_pass(PassArgs a) {
    using Rec = typename P::Rec;
    constexpr int BT = kBlock * T;
    __shared__ Rec s_rec[kTile];
    const int64_t U = a.units, C = a.chunks, G = gridDim.x;
    const int64_t u0 = unit_begin(blockIdx.x, U, G), u1 = unit_begin(blockIdx.x + 1, U, G);
    if (u0 >= u1) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const bool excl = a.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    Tgt<P, T> t;
    bool active = false;
    int64_t tbk = -1;
    double acc[T][P::NACC];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int c = 0; c < P::NACC; ++c) acc[k][c] = 0.0;

    int64_t ub = u0 / C, c = u0 % C;
    for (int64_t u = u0; u < u1; ++u) {
        __syncthreads();
        if (ub != tbk) {
            if (tbk >= 0) flush<P, T>(a, tbk, wave, lane, acc);
            tbk = ub;
            const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
            active = tb < a.n_trg;
            load_tgt<P, T>(a, active ? tb : 0, lane, t);
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int q = 0; q < P::NACC; ++q) acc[k][q] = 0.0;
        }
        // the chunk goes straight to LDS: a record held in registers across
        // the loop below would be spilled
        s_rec[threadIdx.x] = rec[c * kTile + threadIdx.x];
        __syncthreads();
        int64_t cn = c + 1, ubn = ub;
        if (cn == C) { cn = 0; ++ubn; }
        if (active) {
            uint32_t flags = 0;
#pragma unroll 1
            for (int s = 0; s < 4; ++s) {
                const SubMeta m = a.meta[c * 4 + s];
                if (m.count == 0) continue;
                if (needs_near<P, T>(t, m, excl)) {
                    flags |= 1u << s;
                    continue;
                }
                const Rec* base = s_rec + s * kSub;
#pragma unroll 2
                for (int j = 0; j < kSub; ++j) {
                    const Rec sr = base[j];
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        P::template pair<false>(sr, t.x[k], t.y[k], t.z[k], t.v[k], false, acc[k]);
                }
            }
            if (lane == 0) a.flags[(tbk * 4 + wave) * C + c] = (uint8_t)flags;
        }
        c = cn;
        ub = ubn;
    }
    flush<P, T>(a, tbk, wave, lane, acc);
}

template <class P, int T>
__global__ __launch_bounds__(kBlock) void near_pass(PassArgs a) {
    using Rec = typename P::Rec;
    constexpr int BT = kBlock * T;
    // each wave stages its current sub-tile in its own slice (read back by
    // broadcast; only that wave touches it, and a wave's LDS operations
    // complete in order, so no workgroup barrier is needed)
    __shared__ Rec s_src[4][kSub];
    __shared__ int32_t s_grp[4][kSub];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t tbk = blockIdx.x, C = a.chunks;
    const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
    if (tb >= a.n_trg) return;                 // no barriers below
    const bool excl = a.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    Tgt<P, T> t;
    load_tgt<P, T>(a, tb, lane, t);
    double acc[T][P::NACC];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int q = 0; q < P::NACC; ++q) acc[k][q] = 0.0;
    const uint8_t* fl = a.flags + (tbk * 4 + wave) * C;
    for_each_flagged(fl, C, lane, (int)blockIdx.y, [&](int64_t sub) {
        s_src[wave][lane] = rec[sub * kSub + lane];
        s_grp[wave][lane] = a.grp[sub * kSub + lane];
        __builtin_amdgcn_wave_barrier();
#pragma unroll 2
        for (int j = 0; j < kSub; ++j) {
            const Rec sr = s_src[wave][j];
            const int32_t gs = s_grp[wave][j];
#pragma unroll
            for (int k = 0; k < T; ++k)
                P::template pair<true>(sr, t.x[k], t.y[k], t.z[k], t.v[k], excl && gs == t.g[k], acc[k]);
        }
        __builtin_amdgcn_wave_barrier();   // reads of this sub-tile precede the next writes
    });
    const int64_t np = (int64_t)gridDim.x * BT;
    double* part = a.near_part + (int64_t)blockIdx.y * P::NACC * np;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t gi = tbk * BT + wave * (kWave * T) + k * kWave + lane;
#pragma unroll
        for (int q = 0; q < P::NACC; ++q) part[q * np + gi] = acc[k][q];
    }
}

template <class P, int T>
__global__ __launch_bounds__(kBlock) void reduce(PassArgs a, int64_t grid, int64_t np) {
    constexpr int BT = kBlock * T;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n_trg) return;
    const int64_t tbk = i / BT, li = i % BT;
    const int64_t b0 = unit_owner(tbk * a.chunks, a.units, grid);
    const int64_t b1 = unit_owner((tbk + 1) * a.chunks - 1, a.units, grid);
    double s[P::NACC];
#pragma unroll
    for (int q = 0; q < P::NACC; ++q) s[q] = 0.0;
    for (int64_t b = b0; b <= b1; ++b) {
        const double* seg = a.part + (b + tbk) * P::NACC * BT;
#pragma unroll
        for (int q = 0; q < P::NACC; ++q) s[q] += seg[q * BT + li];
    }
    for (int sl = 0; sl < kNearSlices; ++sl)
#pragma unroll
        for (int q = 0; q < P::NACC; ++q) s[q] += a.near_part[(sl * P::NACC + q) * np + i];
    P::store(a, i, s);
}

// ---------------------------------------------------------------------------
// host side: plan and launch one pass
// ---------------------------------------------------------------------------
struct PassPlan {
    int64_t n_src_pad, n_sub, chunks, blocks_x, units, grid;
    size_t off_rec, off_grp, off_meta, off_part, off_near, off_flags, total;
};

template <class P, int T>
PassPlan plan_pass(int64_t n_src, int64_t n_trg, int resident) {
    PassPlan p{};
    p.n_src_pad = ceil_div(n_src, kTile) * kTile;
    p.n_sub = p.n_src_pad / kSub;
    p.chunks = p.n_src_pad / kTile;
    p.blocks_x = ceil_div(n_trg, (int64_t)kBlock * T);
    p.units = p.chunks * p.blocks_x;
    p.grid = std::max<int64_t>(1, std::min<int64_t>(std::max(1, resident), p.units));
    const size_t bt = (size_t)kBlock * T;
    size_t off = 0;
    p.off_rec = off;
    off = align_up(off + (size_t)p.n_src_pad * sizeof(typename P::Rec), 256);
    p.off_grp = off;
    off = align_up(off + (size_t)p.n_src_pad * sizeof(int32_t), 256);
    p.off_meta = off;
    off = align_up(off + (size_t)p.n_sub * sizeof(SubMeta), 256);
    p.off_part = off;
    off = align_up(off + (size_t)(p.grid + p.blocks_x) * P::NACC * bt * sizeof(double), 256);
    p.off_near = off;
    off = align_up(off + (size_t)kNearSlices * p.blocks_x * P::NACC * bt * sizeof(double), 256);
    p.off_flags = off;
    off = align_up(off + (size_t)p.blocks_x * 4 * (size_t)p.chunks, 256);
    p.total = off;
    return p;
}

template <class P, int T, int W>
int resident_blocks(int n_cu) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, main_pass<P, T, W>, kBlock, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb * n_cu;
}

// Runs prep, main, near and reduce on `stream`; a.n_src and a.n_trg > 0.
template <class P, int T, int W>
hipError_t run_pass(PassArgs a, const PassPlan& p, void* ws, hipStream_t stream,
                    const KernelTimer& timer) {
    char* base = static_cast<char*>(ws);
    a.rec = base + p.off_rec;
    a.grp = reinterpret_cast<int32_t*>(base + p.off_grp);
    a.meta = reinterpret_cast<SubMeta*>(base + p.off_meta);
    a.part = reinterpret_cast<double*>(base + p.off_part);
    a.near_part = reinterpret_cast<double*>(base + p.off_near);
    a.flags = reinterpret_cast<uint8_t*>(base + p.off_flags);
    a.chunks = p.chunks;
    a.units = p.units;
    prep<P><<<dim3((unsigned)(p.n_src_pad / kBlock)), dim3(kBlock), 0, stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (timer.on()) (void)hipEventRecord(timer.start, stream);
    main_pass<P, T, W><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (timer.on()) (void)hipEventRecord(timer.stop, stream);
    if (e != hipSuccess) return e;
    near_pass<P, T><<<dim3((unsigned)p.blocks_x, kNearSlices), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce<P, T><<<dim3((unsigned)ceil_div(a.n_trg, kBlock)), dim3(kBlock), 0, stream>>>(
        a, p.grid, p.blocks_x * (int64_t)kBlock * T);
    return hipGetLastError();
}

}  // namespace ps
}  // namespace stokes
