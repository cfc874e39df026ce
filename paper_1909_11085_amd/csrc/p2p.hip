// Leaf-to-leaf (P2P) sums: the near-field part of the FMM evaluation of the
// paper's Sec. 3.1 ("Far evaluation"), where every target leaf sums the
// single- or double-layer kernel over the sources of the leaves in its
// interaction list, in one launch over all the (uneven) lists.
//
// Design (gfx950):
//   * work items: each target leaf cut into 64-target items, sorted by their
//     estimated cost (largest first, for balance).  Two ways in: a plan built
//     once from host arrays (validated and sorted on the host), or device
//     arrays per call, validated and turned into sorted items on the device
//     (a count, a prefix sum, cost keys, a radix sort), with no host round
//     trip; both give the same order.
//   * prep (one wave per leaf, per evaluation): the leaf's box centre and
//     radius, then a packed record per source; mixed precision stores each
//     source's offset from its leaf centre as a float32 high part and residue.
//   * sum: one wave per work item.  An item of n <= 64 targets gives each
//     target R = min(16, 64/n) lanes, and lane phase h takes every R-th source
//     (so small leaves still fill the wave); the R partial sums are added in a
//     fixed order at the end.  The sources of each listed leaf are staged
//     through LDS, up to 128 at a time, and sorted on the way in by what
//     each needs: sources of a group that every target of the item shares
//     are dropped (the same-group rule excludes them all); sources within
//     the near limit of the targets' box are "careful"; sources of a group
//     that some targets share are "masked"; the rest are "clean".  Clean
//     sources run an unmasked loop (float32 offsets in mixed precision,
//     exactly as the direct sums' fast path), masked ones the same loop with
//     the same-group mask (and, in FP64, the zero-distance mask), careful
//     ones (mixed) r = (x_hi - y_hi) + (x_lo - y_lo) with the same-group
//     mask and the pairs inside the near radius evaluated in float64.
#include <float.h>
#include <limits.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/stokes_mi355x.h"
#include "p2p.hpp"
#include "spatial.hpp"

struct stokes_p2p_plan {
    int device;
    int32_t n_leaves;
    int64_t n_src, n_trg, n_ulist, n_items, pairs;
    int64_t* d_src_ofs;      // device copies
    int64_t* d_trg_ofs;
    int64_t* d_ulist_ofs;
    int32_t* d_ulist;
    int32_t* d_items;        // (leaf, chunk) pairs, largest pair count first
};

namespace stokes {
namespace {

constexpr int kP2PTile = 128;    // sources staged per LDS step (two batches of 64)
constexpr int kMaxRep = 16;      // lanes per target at most
constexpr int kMaxTGroups = 8;   // distinct target groups tracked per item
static_assert(kP2PTile % kWave == 0, "staging classifies a tile in batches of one wave");

// src: the source's index within its leaf (staging reorders sources)
struct alignas(16) P2PSL32 { float hx, hy, hz, lx, ly, lz, qx, qy, qz, t2; int32_t g, src; };
struct alignas(16) P2PDL32 {
    float hx, hy, hz, lx, ly, lz, qx, qy, qz, nx, ny, nz, t2;
    int32_t g, src;
    float pad;
};

template <int KT, int MIXED> struct P2PRec;
template <> struct P2PRec<0, 0> { using type = SrcSL64; };
template <> struct P2PRec<1, 0> { using type = SrcDL64; };
template <> struct P2PRec<0, 1> { using type = P2PSL32; };
template <> struct P2PRec<1, 1> { using type = P2PDL32; };
// kernels 2 .. 5: the adjoint sums, float64 only (the pair forms at pair64)
template <> struct P2PRec<2, 0> { using type = SrcSL64; };
template <> struct P2PRec<3, 0> { using type = SrcDL64; };
template <> struct P2PRec<4, 0> { using type = SrcSL64; };
template <> struct P2PRec<5, 0> { using type = SrcSL64; };
// kernels whose source records carry a normal
template <int KT> constexpr bool kSrcNormal = KT == 1 || KT == 3;

struct P2PArgs {
    SumInputs in;
    const int64_t* src_ofs;
    const int64_t* trg_ofs;
    const int64_t* ulist_ofs;
    const int32_t* ulist;
    const int32_t* items;
    const int64_t* n_items;  // device count of items (device-built layouts), else null: one per workgroup
    const int32_t* status;   // device-built layouts: nonzero when the leaf arrays are malformed, else null
    void* rec;
    int32_t* grp;
    double* leaf_ctr;        // (n_leaves, 4): box centre and half-diagonal
    int32_t n_leaves;
    double* out;
    int accumulate;
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

// One wave per leaf: box centre of its sources, then its packed records.
template <int KT, int MIXED>
__global__ __launch_bounds__(kWave) void p2p_prep(P2PArgs a) {
    using Rec = typename P2PRec<KT, MIXED>::type;
    if (a.status && *a.status) return;
    const int32_t L = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t s0 = a.src_ofs[L], s1 = a.src_ofs[L + 1];
    const int64_t n = a.in.n_src;
    const SumInputs& in = a.in;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int64_t i = s0 + lane; i < s1; i += kWave)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], in.src_xyz[c * n + i]);
            hi[c] = fmax(hi[c], in.src_xyz[c * n + i]);
        }
    double ctr[3], rad2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double l = wmin(lo[c]), h = wmax(hi[c]);
        ctr[c] = s1 > s0 ? 0.5 * (l + h) : 0.0;
        if (s1 > s0) rad2 = __builtin_fma(0.5 * (h - l), 0.5 * (h - l), rad2);
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.leaf_ctr[4 * (int64_t)L + c] = ctr[c];
        a.leaf_ctr[4 * (int64_t)L + 3] = sqrt(rad2);
    }
    for (int64_t i = s0 + lane; i < s1; i += kWave) {
        const double w = in.weight ? in.weight[i] : 1.0;
        double y[3], q[3], nv[3] = {0, 0, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            y[c] = in.src_xyz[c * n + i];
            q[c] = w * in.density[c * n + i];
            if (kSrcNormal<KT>) nv[c] = in.normal[c * n + i];
        }
        int32_t g = in.src_group ? in.src_group[i] : 0;
        double rn = 0.0;
        if (MIXED && in.group_h) {
            if (g >= 0 && g < in.n_groups) rn = in.near_frac * in.group_h[g];
            else q[0] = q[1] = q[2] = __builtin_nan("");
        }
        Rec r;
        if constexpr (MIXED == 0) {
            r.x = y[0]; r.y = y[1]; r.z = y[2];
            r.qx = q[0]; r.qy = q[1]; r.qz = q[2];
            if constexpr (kSrcNormal<KT>) { r.nx = nv[0]; r.ny = nv[1]; r.nz = nv[2]; r.pad = 0.0; }
            a.grp[i] = g;
        } else {
            const double o0 = y[0] - ctr[0], o1 = y[1] - ctr[1], o2 = y[2] - ctr[2];
            r.hx = (float)o0; r.hy = (float)o1; r.hz = (float)o2;
            r.lx = (float)(o0 - (double)r.hx);
            r.ly = (float)(o1 - (double)r.hy);
            r.lz = (float)(o2 - (double)r.hz);
            r.qx = (float)q[0]; r.qy = (float)q[1]; r.qz = (float)q[2];
            if constexpr (KT == 1) { r.nx = (float)nv[0]; r.ny = (float)nv[1]; r.nz = (float)nv[2]; }
            r.t2 = (float)(rn * rn);
            r.g = g;
            r.src = (int32_t)(i - s0);
        }
        reinterpret_cast<Rec*>(a.rec)[i] = r;
    }
}

__device__ __forceinline__ double rinv(double r2, bool skip) {
    const double y0 = skip ? 0.0 : __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y0 * y0, 1.0);
    return __builtin_fma(0.5 * y0, e, y0);
}

// G(r; a, b, c) = [(r.b)(r.c) a + (r.a)(r.c) b + (r.a)(r.b) c]/rho^5
//                 - 5 (r.a)(r.b)(r.c) r/rho^7,
// the gradient in r of (r.a)(r.b)(r.c)/rho^5 (symmetric in a, b, c; even in r),
// added to (ax, ay, az); ri2 = 1/rho^2, ri5 = 1/rho^5.
__device__ __forceinline__ void grad3(double dx, double dy, double dz, double ri2, double ri5, const double (&va)[3],
                                      const double (&vb)[3], const double (&vc)[3], double& ax, double& ay,
                                      double& az) {
    const double ra = __builtin_fma(dx, va[0], __builtin_fma(dy, va[1], dz * va[2]));
    const double rb = __builtin_fma(dx, vb[0], __builtin_fma(dy, vb[1], dz * vb[2]));
    const double rc = __builtin_fma(dx, vc[0], __builtin_fma(dy, vc[1], dz * vc[2]));
    const double bc = rb * rc * ri5, ac = ra * rc * ri5, ab = ra * rb * ri5;
    const double cr = -5.0 * ra * bc * ri2;
    ax = __builtin_fma(bc, va[0], __builtin_fma(ac, vb[0], __builtin_fma(ab, vc[0], __builtin_fma(cr, dx, ax))));
    ay = __builtin_fma(bc, va[1], __builtin_fma(ac, vb[1], __builtin_fma(ab, vc[1], __builtin_fma(cr, dy, ay))));
    az = __builtin_fma(bc, va[2], __builtin_fma(ac, vb[2], __builtin_fma(ab, vc[2], __builtin_fma(cr, dz, az))));
}

// KT 0: q/rho + r (r.q)/rho^3; KT 1: r (r.n)(r.q)/rho^5; KT 2: the gradient in
// r of a.S(r)b times 8 pi mu, with a = tv (the target's vector) and b = q:
//   K(r; a, b) = [(r.b) a + (r.a) b - (a.b) r]/rho^3 - 3 (r.a)(r.b) r/rho^5;
// KT 3: G(r; n, q, tv) (the double layer's gradient, source normal n);
// KT 4: r (r.tv)(r.q)/rho^5 (the double-layer form with the normal at the
// target); KT 5: G(r; tv, tv2, q).
template <int KT, bool MASKED>
__device__ __forceinline__ void pair64(const typename P2PRec<KT, 0>::type& s, double x, double y,
                                       double z, const double (&tv)[3], const double (&tv2)[3], bool skip_group,
                                       double& ax, double& ay, double& az) {
    const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double ri = rinv(r2, MASKED && (skip_group || r2 == 0.0));
    const double ri2 = ri * ri;
    const double rq = __builtin_fma(dx, s.qx, __builtin_fma(dy, s.qy, dz * s.qz));
    if constexpr (KT == 2) {
        const double ri3 = ri2 * ri;
        const double ra = __builtin_fma(dx, tv[0], __builtin_fma(dy, tv[1], dz * tv[2]));
        const double ab = __builtin_fma(tv[0], s.qx, __builtin_fma(tv[1], s.qy, tv[2] * s.qz));
        const double sa = rq * ri3, sb = ra * ri3;
        const double cr = -ri3 * __builtin_fma(3.0 * ra * rq, ri2, ab);
        ax = __builtin_fma(sa, tv[0], __builtin_fma(sb, s.qx, __builtin_fma(cr, dx, ax)));
        ay = __builtin_fma(sa, tv[1], __builtin_fma(sb, s.qy, __builtin_fma(cr, dy, ay)));
        az = __builtin_fma(sa, tv[2], __builtin_fma(sb, s.qz, __builtin_fma(cr, dz, az)));
    } else if constexpr (KT == 0) {
        const double c = rq * ri2;
        ax = __builtin_fma(__builtin_fma(c, dx, s.qx), ri, ax);
        ay = __builtin_fma(__builtin_fma(c, dy, s.qy), ri, ay);
        az = __builtin_fma(__builtin_fma(c, dz, s.qz), ri, az);
    } else if constexpr (KT == 3) {
        const double sn[3] = {s.nx, s.ny, s.nz}, sq[3] = {s.qx, s.qy, s.qz};
        grad3(dx, dy, dz, ri2, ri2 * ri2 * ri, sn, sq, tv, ax, ay, az);
    } else if constexpr (KT == 5) {
        const double sq[3] = {s.qx, s.qy, s.qz};
        grad3(dx, dy, dz, ri2, ri2 * ri2 * ri, tv, tv2, sq, ax, ay, az);
    } else if constexpr (KT == 4) {
        const double ra = __builtin_fma(dx, tv[0], __builtin_fma(dy, tv[1], dz * tv[2]));
        const double c = ra * rq * (ri2 * ri2 * ri);
        ax = __builtin_fma(c, dx, ax);
        ay = __builtin_fma(c, dy, ay);
        az = __builtin_fma(c, dz, az);
    } else {
        const double rn = __builtin_fma(dx, s.nx, __builtin_fma(dy, s.ny, dz * s.nz));
        const double c = rn * rq * (ri2 * ri2 * ri);
        ax = __builtin_fma(c, dx, ax);
        ay = __builtin_fma(c, dy, ay);
        az = __builtin_fma(c, dz, az);
    }
}

// float32 pair on offsets from the source leaf's centre, without residues
// (sources outside the near limit); MASKED adds the same-group mask
template <int KT, bool MASKED>
__device__ __forceinline__ void pair32(const typename P2PRec<KT, 1>::type& s, float xs, float ys,
                                       float zs, bool skip, float& bx, float& by, float& bz) {
    const float dx = xs - s.hx, dy = ys - s.hy, dz = zs - s.hz;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float ri = (MASKED && skip) ? 0.0f : __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float rq = __builtin_fmaf(dx, s.qx, __builtin_fmaf(dy, s.qy, dz * s.qz));
    if constexpr (KT == 0) {
        const float c = rq * ri2;
        bx = __builtin_fmaf(__builtin_fmaf(c, dx, s.qx), ri, bx);
        by = __builtin_fmaf(__builtin_fmaf(c, dy, s.qy), ri, by);
        bz = __builtin_fmaf(__builtin_fmaf(c, dz, s.qz), ri, bz);
    } else {
        const float rn = __builtin_fmaf(dx, s.nx, __builtin_fmaf(dy, s.ny, dz * s.nz));
        const float c = rn * rq * (ri2 * ri2 * ri);
        bx = __builtin_fmaf(c, dx, bx);
        by = __builtin_fmaf(c, dy, by);
        bz = __builtin_fmaf(c, dz, bz);
    }
}

// float64 evaluation of one pair from the caller's arrays (near pairs, mixed).
// Out of line (rarely taken) with every argument and the result in registers.
struct Vec3 { double x, y, z; };
template <int KT>
__device__ __noinline__ Vec3 near64(const double* __restrict__ src_xyz, const double* __restrict__ density,
                                    const double* __restrict__ weight, const double* __restrict__ normal,
                                    int64_t ns, int64_t m, double x, double y, double z) {
    const double dx = x - src_xyz[m], dy = y - src_xyz[ns + m], dz = z - src_xyz[2 * ns + m];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return Vec3{0.0, 0.0, 0.0};
    const double w = weight ? weight[m] : 1.0;
    const double qx = w * density[m], qy = w * density[ns + m], qz = w * density[2 * ns + m];
    const double ri = 1.0 / sqrt(r2);
    const double rq = dx * qx + dy * qy + dz * qz;
    if constexpr (KT == 0) {
        const double c = rq * ri * ri;
        return Vec3{(qx + c * dx) * ri, (qy + c * dy) * ri, (qz + c * dz) * ri};
    } else {
        const double rn = dx * normal[m] + dy * normal[ns + m] + dz * normal[2 * ns + m];
        const double c = rn * rq * (ri * ri) * (ri * ri) * ri;
        return Vec3{c * dx, c * dy, c * dz};
    }
}

// Record written into the padding of the clean region: far away, zero strength.
template <typename Rec>
__device__ __forceinline__ Rec pad_record() {
    Rec r{};
    if constexpr (sizeof(r.qx) == 8) {
        r.x = r.y = r.z = kPadPos;
    } else {
        r.hx = r.hy = r.hz = kPadOff;
    }
    return r;
}

// number of set bits of m below this lane
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// CNT (mixed, test-only instantiation): also record each pair's class.
template <int KT, int MIXED, bool CNT = false>
__global__ __launch_bounds__(kWave) void p2p_sum(P2PArgs a) {
    using Rec = typename P2PRec<KT, MIXED>::type;
    constexpr int kSlots = kP2PTile + 2 * kMaxRep;
    // staged sources: clean ones from the front, the others from the back;
    // each region is padded with zero-strength records to R runs of equal
    // length
    __shared__ Rec s_rec[kSlots];
    __shared__ int32_t s_grp[MIXED ? 1 : kSlots];
    if (a.status && *a.status) return;
    if (a.n_items && (int64_t)blockIdx.x >= *a.n_items) return;   // the grid covers the upper bound
    const int lane = threadIdx.x;
    const int32_t L = a.items[2 * blockIdx.x], ch = a.items[2 * blockIdx.x + 1];
    const int64_t t0 = a.trg_ofs[L] + (int64_t)ch * kWave;
    const int nc = (int)min(a.trg_ofs[L + 1] - t0, (int64_t)kWave);   // 1..64 (the plan makes no empty item)
    const int R = min(kMaxRep, kWave / nc);
    const int ti = lane / R, h = lane - ti * R;
    const bool valid = ti < nc;
    const int64_t idx = t0 + (valid ? ti : 0);        // idle lanes mirror target t0
    const int64_t nt = a.in.n_trg;
    const double x = a.in.trg_xyz[idx], y = a.in.trg_xyz[nt + idx], z = a.in.trg_xyz[2 * nt + idx];
    double tv[3] = {0.0, 0.0, 0.0}, tv2[3] = {0.0, 0.0, 0.0};   // kernels 2 .. 5: the target's vectors
    if constexpr (KT >= 2) {
        tv[0] = a.in.trg_vec[idx];
        tv[1] = a.in.trg_vec[nt + idx];
        tv[2] = a.in.trg_vec[2 * nt + idx];
    }
    if constexpr (KT == 5) {
        tv2[0] = a.in.trg_vec2[idx];
        tv2[1] = a.in.trg_vec2[nt + idx];
        tv2[2] = a.in.trg_vec2[2 * nt + idx];
    }
    const int32_t tg = a.in.trg_group ? a.in.trg_group[idx] : 0;
    const bool excl = a.in.excl != 0;

    // the item's target box and its distinct target groups (uniform)
    const double blo[3] = {wmin(x), wmin(y), wmin(z)}, bhi[3] = {wmax(x), wmax(y), wmax(z)};
    int32_t tgl[kMaxTGroups];
#pragma unroll
    for (int q = 0; q < kMaxTGroups; ++q) tgl[q] = 0;
    int ntg = 0;
    bool many_groups = false;
    if (excl) {
        uint64_t rem = __ballot(1);
        while (rem) {                                  // each pass removes at least one lane
            const int first = __builtin_ctzll(rem);
            const int32_t g0 = __builtin_amdgcn_readlane(tg, first);
#pragma unroll
            for (int q = 0; q < kMaxTGroups; ++q)
                if (q == ntg) tgl[q] = g0;
            many_groups |= ntg >= kMaxTGroups;
            ++ntg;
            rem &= ~__ballot(tg == g0);
        }
    }
    const double sext = fmax(fmax(bhi[0] - blo[0], bhi[1] - blo[1]), bhi[2] - blo[2]);

    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t k = a.ulist_ofs[L]; k < a.ulist_ofs[L + 1]; ++k) {
        const int32_t Ls = a.ulist[k];
        const int64_t s0 = a.src_ofs[Ls], ns = a.src_ofs[Ls + 1] - s0;
        const double* lc = a.leaf_ctr + 4 * (int64_t)Ls;
        const double cx = lc[0], cy = lc[1], cz = lc[2], crad = lc[3];
        float xs = 0.f, ys = 0.f, zs = 0.f, xl = 0.f, yl = 0.f, zl = 0.f;
        // mixed: the targets' box relative to this leaf's centre in float32,
        // and a slack above every rounding of the float32 gap test below
        float flo[3] = {0.f, 0.f, 0.f}, fhi[3] = {0.f, 0.f, 0.f}, fslack = 0.f, frad8 = 0.f;
        if constexpr (MIXED != 0) {
            const double hx = x - cx, hy = y - cy, hz = z - cz;
            xs = (float)hx; ys = (float)hy; zs = (float)hz;
            xl = (float)(hx - (double)xs);
            yl = (float)(hy - (double)ys);
            zl = (float)(hz - (double)zs);
            const double cc[3] = {cx, cy, cz};
            double mag = crad;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                flo[q] = (float)(blo[q] - cc[q]);
                fhi[q] = (float)(bhi[q] - cc[q]);
                mag = fmax(mag, fmax(fabs(blo[q] - cc[q]), fabs(bhi[q] - cc[q])));
            }
            fslack = (float)(0x1p-18 * (mag + crad + sext));
            frad8 = (float)(0.125 * crad);
        }
        for (int64_t b = 0; b < ns; b += kP2PTile) {
            const int nb = (int)((ns - b) < kP2PTile ? (ns - b) : kP2PTile);
            // sort the tile's sources into LDS as they arrive (batches of 64):
            //   clean (front): no group shared with the item's targets, outside
            //     the near limit of their box: unmasked loop;
            //   back: a group shared with some targets (same loop plus the
            //     same-group mask; FP64 also masks zero distance), or (mixed)
            //     within the near limit: residues and near test.  The back
            //     region takes the careful loop if it holds any of the latter;
            //   dropped: a group that every target of the item shares.
            __syncthreads();                           // previous readers are done
            int n_clean = 0, n_back = 0;
            bool any_close = false;
            for (int i0 = 0; i0 < nb; i0 += kWave) {
                const int i = i0 + lane;
                const bool in = i < nb;
                const int64_t si = s0 + b + (in ? i : 0);     // nb >= 1: index 0 is a real source
                const Rec r = rec[si];
                int32_t g;
                bool close;
                if constexpr (MIXED == 0) {
                    g = a.grp[si];
                    // coincident points are possible only inside the targets' box
                    const double gx = fmax(fmax(blo[0] - r.x, r.x - bhi[0]), 0.0);
                    const double gy = fmax(fmax(blo[1] - r.y, r.y - bhi[1]), 0.0);
                    const double gz = fmax(fmax(blo[2] - r.z, r.z - bhi[2]), 0.0);
                    close = __builtin_fma(gx, gx, __builtin_fma(gy, gy, gz * gz)) <= 1e-200;
                } else {
                    g = r.g;
                    // gap from the targets' box in float32 on leaf-centred
                    // offsets; the limit is the near radius with margin, or an
                    // eighth of the leaf radius (which bounds the float32 offset
                    // error of the unmasked formula to about 20 ulp per pair),
                    // plus the slack
                    const float gx = fmaxf(fmaxf(flo[0] - r.hx, r.hx - fhi[0]), 0.f);
                    const float gy = fmaxf(fmaxf(flo[1] - r.hy, r.hy - fhi[1]), 0.f);
                    const float gz = fmaxf(fmaxf(flo[2] - r.hz, r.hz - fhi[2]), 0.f);
                    const float gap2 = __builtin_fmaf(gx, gx, __builtin_fmaf(gy, gy, gz * gz));
                    const float lim = fmaxf(1.001f * __builtin_amdgcn_sqrtf(r.t2), frad8) + fslack;
                    close = !(gap2 > lim * lim);
                }
                bool shared = false;
                if (excl) {
                    shared = many_groups;
#pragma unroll
                    for (int q = 0; q < kMaxTGroups; ++q) shared |= (q < ntg) && g == tgl[q];
                }
                const bool keep = in && !(excl && ntg == 1 && g == tgl[0]);
                if constexpr (CNT) {
                    if (in && !keep)                   // every target of the item shares its group
                        for (int q = 0; q < nc; ++q)
                            atomicAdd(a.in.pair_class + (t0 + q) * a.in.n_src + si, kPairSkip);
                }
                const bool back = close || shared;
                const uint64_t mf = __ballot(keep && !back), mk = __ballot(keep && back);
                if (MIXED && __ballot(keep && close)) any_close = true;
                if (keep) {
                    const int pos = back ? kSlots - 1 - (n_back + lanes_below(mk)) : n_clean + lanes_below(mf);
                    s_rec[pos] = r;
                    if constexpr (MIXED == 0) s_grp[pos] = g;
                }
                n_clean += __popcll(mf);
                n_back += __popcll(mk);
            }
            const int m_clean = (n_clean + R - 1) / R, m_back = (n_back + R - 1) / R;
            const int n_clean_pad = m_clean * R, n_back_pad = m_back * R;
            const int kb = kSlots - n_back_pad;        // back region [kb, kSlots), pad first
            if (lane < n_clean_pad - n_clean) s_rec[n_clean + lane] = pad_record<Rec>();
            if (lane < n_back_pad - n_back) {
                s_rec[kb + lane] = pad_record<Rec>();
                if constexpr (MIXED == 0) s_grp[kb + lane] = 0;
            }
            __syncthreads();

            // phase h takes the h-th of the R runs of each region
            const Rec* pc = s_rec + h * m_clean;
            const Rec* pb = s_rec + kb + h * m_back;
            if constexpr (MIXED == 0) {
                const int32_t* gbk = s_grp + kb + h * m_back;
#pragma unroll 4
                for (int j = 0; j < m_clean; ++j) pair64<KT, false>(pc[j], x, y, z, tv, tv2, false, ax, ay, az);
#pragma unroll 2
                for (int j = 0; j < m_back; ++j)
                    pair64<KT, true>(pb[j], x, y, z, tv, tv2, excl && gbk[j] == tg, ax, ay, az);
            } else {
                float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll 4
                for (int j = 0; j < m_clean; ++j) pair32<KT, false>(pc[j], xs, ys, zs, false, bx, by, bz);
                // CNT: staged slots [0, n_clean) and [kb + back padding, kSlots) hold real sources
                const int back_real = kb + (n_back_pad - n_back);
                if constexpr (CNT) {
                    if (valid)
                        for (int j = 0; j < m_clean; ++j)
                            if (h * m_clean + j < n_clean)
                                atomicAdd(a.in.pair_class + idx * a.in.n_src + s0 + pc[j].src, kPairF32);
                }
                if (!any_close) {
#pragma unroll 2
                    for (int j = 0; j < m_back; ++j) {
                        const Rec sr = pb[j];
                        pair32<KT, true>(sr, xs, ys, zs, excl && sr.g == tg, bx, by, bz);
                        if constexpr (CNT) {
                            if (valid && kb + h * m_back + j >= back_real)
                                atomicAdd(a.in.pair_class + idx * a.in.n_src + s0 + sr.src,
                                          (excl && sr.g == tg) ? kPairSkip : kPairF32);
                        }
                    }
                } else {
                    // residues, near test, float64 near pairs
                    for (int j = 0; j < m_back; ++j) {
                        const Rec sr = pb[j];
                        const float dx = (xs - sr.hx) + (xl - sr.lx);
                        const float dy = (ys - sr.hy) + (yl - sr.ly);
                        const float dz = (zs - sr.hz) + (zl - sr.lz);
                        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                        const bool excluded = excl && sr.g == tg;
                        const bool near = r2 <= sr.t2;
                        const float ri = (excluded || near) ? 0.0f : __builtin_amdgcn_rsqf(r2);
                        const float ri2 = ri * ri;
                        const float rq = __builtin_fmaf(dx, sr.qx, __builtin_fmaf(dy, sr.qy, dz * sr.qz));
                        if constexpr (KT == 0) {
                            const float c = rq * ri2;
                            bx = __builtin_fmaf(__builtin_fmaf(c, dx, sr.qx), ri, bx);
                            by = __builtin_fmaf(__builtin_fmaf(c, dy, sr.qy), ri, by);
                            bz = __builtin_fmaf(__builtin_fmaf(c, dz, sr.qz), ri, bz);
                        } else {
                            const float rn = __builtin_fmaf(dx, sr.nx, __builtin_fmaf(dy, sr.ny, dz * sr.nz));
                            const float c = rn * rq * (ri2 * ri2 * ri);
                            bx = __builtin_fmaf(c, dx, bx);
                            by = __builtin_fmaf(c, dy, by);
                            bz = __builtin_fmaf(c, dz, bz);
                        }
                        if (near && !excluded) {
                            const Vec3 v = near64<KT>(a.in.src_xyz, a.in.density, a.in.weight, a.in.normal,
                                                      a.in.n_src, s0 + sr.src, x, y, z);
                            ax += v.x;
                            ay += v.y;
                            az += v.z;
                        }
                        if constexpr (CNT) {
                            if (valid && kb + h * m_back + j >= back_real) {
                                // near64 takes nothing at zero distance (float64)
                                const int64_t nsrc = a.in.n_src, si = s0 + sr.src;
                                const bool zero = x == a.in.src_xyz[si] && y == a.in.src_xyz[nsrc + si] &&
                                                  z == a.in.src_xyz[2 * nsrc + si];
                                atomicAdd(a.in.pair_class + idx * nsrc + si,
                                          excluded ? kPairSkip : !near ? kPairF32 : zero ? kPairSkip : kPairF64);
                            }
                        }
                    }
                }
                ax += (double)bx;
                ay += (double)by;
                az += (double)bz;
            }
        }
    }
    // add the R phase partials of each target in a fixed order
    if (R > 1) {
        static_assert(sizeof(s_rec) >= 3 * kWave * sizeof(double), "reduction reuses the staging array");
        double* s_red = reinterpret_cast<double*>(s_rec);
        __syncthreads();                               // last tile's readers are done
        s_red[lane] = ax;
        s_red[kWave + lane] = ay;
        s_red[2 * kWave + lane] = az;
        __syncthreads();
        if (valid && h == 0) {                         // lanes ti*R .. ti*R + R - 1 < nc*R <= 64
            for (int q = 1; q < R; ++q) {
                ax += s_red[lane + q];
                ay += s_red[kWave + lane + q];
                az += s_red[2 * kWave + lane + q];
            }
        }
    }
    if (valid && h == 0) {
        const double p = a.in.pref;
        const int64_t o = a.in.trg_perm ? (int64_t)a.in.trg_perm[idx] : idx;
        if (a.accumulate) {
            a.out[o] += p * ax;
            a.out[nt + o] += p * ay;
            a.out[2 * nt + o] += p * az;
        } else {
            a.out[o] = p * ax;
            a.out[nt + o] = p * ay;
            a.out[2 * nt + o] = p * az;
        }
    }
}

size_t rec_size(int kernel, int mixed) {
    if (kernel == 2 || kernel == 4 || kernel == 5) return sizeof(SrcSL64);
    if (kernel == 3) return sizeof(SrcDL64);
    if (!mixed) return kernel == 0 ? sizeof(P2PRec<0, 0>::type) : sizeof(P2PRec<1, 0>::type);
    return kernel == 0 ? sizeof(P2PRec<0, 1>::type) : sizeof(P2PRec<1, 1>::type);
}

struct P2PLayout {
    size_t off_rec, off_grp, off_ctr;
    // device-built items (per-call leaf arrays)
    int64_t max_items;
    SortLayout sort;
    size_t off_status, off_cnt, off_listed, off_scan, off_nitems, off_items, off_keys, off_vals, off_sorted,
        off_sort, total;
};

// Upper bound of the work items: every leaf adds at most one partial chunk to
// the full ones.
int64_t max_p2p_items(int64_t n_trg, int32_t n_leaves) {
    return (n_trg + kWave - 1) / kWave + std::min<int64_t>(n_trg, n_leaves);
}

P2PLayout p2p_layout(int kernel, int mixed, int64_t n_src, int64_t n_trg, int32_t n_leaves) {
    P2PLayout l{};
    size_t off = 0;
    l.off_rec = off;
    off = align_up(off + (size_t)std::max<int64_t>(n_src, 1) * rec_size(kernel, mixed), 256);
    l.off_grp = off;
    off = align_up(off + (size_t)std::max<int64_t>(n_src, 1) * sizeof(int32_t), 256);
    l.off_ctr = off;
    off = align_up(off + (size_t)std::max(n_leaves, 1) * 4 * sizeof(double), 256);
    const int64_t nl = std::max(n_leaves, 1);
    l.max_items = std::max<int64_t>(max_p2p_items(n_trg, n_leaves), 1);
    l.sort = sort_layout(l.max_items);
    l.off_status = off;
    off = align_up(off + sizeof(int32_t), 256);
    l.off_cnt = off;
    off = align_up(off + (size_t)(nl + 1) * sizeof(int64_t), 256);
    l.off_listed = off;
    off = align_up(off + (size_t)nl * sizeof(int64_t), 256);
    l.off_scan = off;
    off = align_up(off + (size_t)scan_tmp_count(nl) * sizeof(int64_t), 256);
    l.off_nitems = off;
    off = align_up(off + sizeof(int64_t), 256);
    l.off_items = off;
    off = align_up(off + (size_t)l.max_items * 2 * sizeof(int32_t), 256);
    l.off_keys = off;
    off = align_up(off + (size_t)l.max_items * sizeof(uint64_t), 256);
    l.off_vals = off;
    off = align_up(off + (size_t)l.max_items * sizeof(int32_t), 256);
    l.off_sorted = off;
    off = align_up(off + (size_t)l.max_items * 2 * sizeof(int32_t), 256);
    l.off_sort = off;
    off = align_up(off + l.sort.total, 256);
    l.total = off;
    return l;
}

// What the sum kernels take from a leaf layout: its device arrays and items.
struct P2PItems {
    const int64_t *src_ofs, *trg_ofs, *ulist_ofs;
    const int32_t* ulist;
    const int32_t* items;
    const int64_t* n_items;   // device count, or null (then grid == the item count)
    const int32_t* status;    // or null
    int32_t n_leaves;
    int64_t grid;             // workgroups of the sum
};

template <int KT, int MIXED>
hipError_t run_p2p(P2PArgs a, const P2PItems& it, void* ws, hipStream_t stream, const KernelTimer& timer) {
    const P2PLayout l = p2p_layout(KT, MIXED, a.in.n_src, a.in.n_trg, it.n_leaves);
    char* base = static_cast<char*>(ws);
    a.src_ofs = it.src_ofs;
    a.trg_ofs = it.trg_ofs;
    a.ulist_ofs = it.ulist_ofs;
    a.ulist = it.ulist;
    a.items = it.items;
    a.n_items = it.n_items;
    a.status = it.status;
    a.n_leaves = it.n_leaves;
    a.rec = base + l.off_rec;
    a.grp = reinterpret_cast<int32_t*>(base + l.off_grp);
    a.leaf_ctr = reinterpret_cast<double*>(base + l.off_ctr);
    if (it.n_leaves > 0) {
        p2p_prep<KT, MIXED><<<dim3((unsigned)it.n_leaves), dim3(kWave), 0, stream>>>(a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (it.grid == 0) return hipSuccess;
    if (timer.on()) (void)hipEventRecord(timer.start, stream);
    if constexpr (MIXED != 0) {
        if (a.in.pair_class)
            p2p_sum<KT, MIXED, true><<<dim3((unsigned)it.grid), dim3(kWave), 0, stream>>>(a);
        else
            p2p_sum<KT, MIXED><<<dim3((unsigned)it.grid), dim3(kWave), 0, stream>>>(a);
    } else {
        p2p_sum<KT, MIXED><<<dim3((unsigned)it.grid), dim3(kWave), 0, stream>>>(a);
    }
    hipError_t e = hipGetLastError();
    if (timer.on()) (void)hipEventRecord(timer.stop, stream);
    return e;
}

template <int KT, int MIXED>
hipError_t run_p2p_typed(const SumInputs& in, const P2PItems& it, double* out, int accumulate, void* ws,
                         hipStream_t stream, const KernelTimer& timer) {
    P2PArgs a{};
    a.in = in;
    a.out = out;
    a.accumulate = accumulate;
    return run_p2p<KT, MIXED>(a, it, ws, stream, timer);
}

hipError_t run_p2p_any(const SumInputs& in, const P2PItems& it, double* out, int accumulate, void* ws,
                       hipStream_t stream, const KernelTimer& timer) {
    if (in.kernel == 2) return run_p2p_typed<2, 0>(in, it, out, accumulate, ws, stream, timer);
    if (in.kernel == 3) return run_p2p_typed<3, 0>(in, it, out, accumulate, ws, stream, timer);
    if (in.kernel == 4) return run_p2p_typed<4, 0>(in, it, out, accumulate, ws, stream, timer);
    if (in.kernel == 5) return run_p2p_typed<5, 0>(in, it, out, accumulate, ws, stream, timer);
    if (in.kernel == 0)
        return in.mixed ? run_p2p_typed<0, 1>(in, it, out, accumulate, ws, stream, timer)
                        : run_p2p_typed<0, 0>(in, it, out, accumulate, ws, stream, timer);
    return in.mixed ? run_p2p_typed<1, 1>(in, it, out, accumulate, ws, stream, timer)
                    : run_p2p_typed<1, 0>(in, it, out, accumulate, ws, stream, timer);
}

// ---------------------------------------------------------------------------
// work items from device leaf arrays
// ---------------------------------------------------------------------------
constexpr int kP2PThreads = 256;
constexpr int kItemKeyBits = 16;
constexpr uint64_t kItemKeyTop = (1ull << kItemKeyBits) - 1;

// A cost on a log scale in 16 bits (a float32's exponent and top 10 mantissa
// bits): non-decreasing in the cost, steps of 2^-10 of it, so two radix passes
// order the items.
__device__ __forceinline__ uint64_t cost_code(uint64_t cost) {
    const uint32_t b = __float_as_uint((float)cost);   // cost >= 1: exponent field >= 127
    return (uint64_t)((b >> 13) - (127u << 10));
}

__global__ __launch_bounds__(kP2PThreads) void p2p_set_i32(int32_t* p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}
__global__ __launch_bounds__(kP2PThreads) void p2p_copy_i32(const int32_t* from, int32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = *from;
}

// The leaf arrays' contract: each offset array starts at 0, never decreases
// and ends at its total; every list entry names a leaf.  Any breach sets
// *status.
__global__ __launch_bounds__(kP2PThreads) void p2p_csr_check(const int64_t* __restrict__ so,
                                                             const int64_t* __restrict__ to,
                                                             const int64_t* __restrict__ uo,
                                                             const int32_t* __restrict__ ul, int32_t nl,
                                                             int64_t ns, int64_t nt, int64_t nu,
                                                             int32_t* __restrict__ status) {
    const int64_t n = std::max<int64_t>((int64_t)nl + 1, nu);
    for (int64_t i = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kP2PThreads) {
        bool bad = false;
        if (i <= nl) {
            const int64_t* o[3] = {so, to, uo};
            const int64_t tot[3] = {ns, nt, nu};
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (i == 0 && o[q][0] != 0) bad = true;
                if (i == nl && o[q][nl] != tot[q]) bad = true;
                if (i < nl && o[q][i + 1] < o[q][i]) bad = true;
            }
        }
        if (i < nu && (ul[i] < 0 || ul[i] >= nl)) bad = true;
        if (bad) atomicOr(status, 1);
    }
}

// Per leaf: its 64-target chunks and the sources its list holds (0 chunks
// when the arrays are malformed).
__global__ __launch_bounds__(kP2PThreads) void p2p_csr_count(const int64_t* __restrict__ so,
                                                             const int64_t* __restrict__ to,
                                                             const int64_t* __restrict__ uo,
                                                             const int32_t* __restrict__ ul, int32_t nl,
                                                             const int32_t* __restrict__ status,
                                                             int64_t* __restrict__ cnt, int64_t* __restrict__ listed) {
    const bool ok = *status == 0;
    for (int64_t L = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; L < nl; L += (int64_t)gridDim.x * kP2PThreads) {
        int64_t c = 0, s = 0;
        if (ok) {
            c = (to[L + 1] - to[L] + kWave - 1) / kWave;
            for (int64_t k = uo[L]; k < uo[L + 1]; ++k) s += so[ul[k] + 1] - so[ul[k]];
        }
        cnt[L] = c;
        listed[L] = s;
    }
}

// Every slot gets the top key (unused slots sort last) and its own index.
__global__ __launch_bounds__(kP2PThreads) void p2p_item_slots(int64_t max_items, uint64_t* __restrict__ keys,
                                                              int32_t* __restrict__ vals) {
    for (int64_t k = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; k < max_items;
         k += (int64_t)gridDim.x * kP2PThreads) {
        keys[k] = kItemKeyTop;
        vals[k] = (int32_t)k;
    }
}

// The items of each leaf, in leaf and chunk order, with their cost keys: the
// pair loop of an n-target item runs s/R steps over the s listed sources,
// R = min(16, 64/n); the key is the inverted log-scale code of that cost, so
// that an ascending stable sort puts the largest first (the host-built plan's
// order up to costs within 2^-10 of each other, which keep leaf order).  The
// order only schedules the items: each target's sum is one item's.
__global__ __launch_bounds__(kP2PThreads) void p2p_csr_items(const int64_t* __restrict__ to,
                                                             const int64_t* __restrict__ cofs,
                                                             const int64_t* __restrict__ listed, int32_t nl,
                                                             int64_t max_items, int32_t* __restrict__ items,
                                                             uint64_t* __restrict__ keys) {
    for (int64_t L = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; L < nl; L += (int64_t)gridDim.x * kP2PThreads) {
        const int64_t nt = to[L + 1] - to[L], s = listed[L];
        for (int64_t c = 0; c * kWave < nt; ++c) {
            const int64_t k = cofs[L] + c;
            if (k >= max_items) break;
            const int64_t n_c = std::min<int64_t>(kWave, nt - c * kWave);
            const int64_t rep = std::min<int64_t>(kMaxRep, kWave / n_c);
            const uint64_t cost = (uint64_t)(s * 64 / rep + s + 1);
            items[2 * k] = (int32_t)L;
            items[2 * k + 1] = (int32_t)c;
            keys[k] = kItemKeyTop - 1 - std::min<uint64_t>(cost_code(cost), kItemKeyTop - 1);
        }
    }
}

__global__ __launch_bounds__(kP2PThreads) void p2p_item_order(const int32_t* __restrict__ items,
                                                              const int32_t* __restrict__ order,
                                                              const int64_t* __restrict__ n_items,
                                                              int32_t* __restrict__ sorted) {
    const int64_t count = *n_items;
    for (int64_t k = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; k < count; k += (int64_t)gridDim.x * kP2PThreads) {
        sorted[2 * k] = items[2 * order[k]];
        sorted[2 * k + 1] = items[2 * order[k] + 1];
    }
}

// Malformed leaf arrays: every output component becomes NaN.
__global__ __launch_bounds__(kP2PThreads) void p2p_poison(const int32_t* __restrict__ status, double* __restrict__ out,
                                                          int64_t n) {
    if (*status == 0) return;
    for (int64_t i = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kP2PThreads)
        out[i] = __builtin_nan("");
}

unsigned p2p_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kP2PThreads - 1) / kP2PThreads, 4096));
}

}  // namespace

size_t p2p_workspace_bytes(int kernel, int mixed, int64_t n_src, int64_t n_trg, int32_t n_leaves) {
    if (n_src <= 0 || n_trg <= 0) return 0;
    return p2p_layout(kernel, mixed, n_src, n_trg, n_leaves).total;
}

hipError_t launch_p2p(const SumInputs& in, const stokes_p2p_plan* plan, double* out, int accumulate,
                      void* ws, hipStream_t stream, const KernelTimer& timer) {
    const P2PItems it{plan->d_src_ofs, plan->d_trg_ofs, plan->d_ulist_ofs, plan->d_ulist, plan->d_items,
                      nullptr, nullptr, plan->n_leaves, plan->n_items};
    return run_p2p_any(in, it, out, accumulate, ws, stream, timer);
}

hipError_t launch_p2p_csr(const SumInputs& in, int32_t n_leaves, const int64_t* src_ofs, const int64_t* trg_ofs,
                          const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist, double* out,
                          int accumulate, void* ws, hipStream_t st, const KernelTimer& timer, bool check,
                          const int32_t* ext_status) {
    const P2PLayout l = p2p_layout(in.kernel, in.mixed, in.n_src, in.n_trg, n_leaves);
    char* base = static_cast<char*>(ws);
    int32_t* status = reinterpret_cast<int32_t*>(base + l.off_status);
    int64_t* cnt = reinterpret_cast<int64_t*>(base + l.off_cnt);
    int64_t* listed = reinterpret_cast<int64_t*>(base + l.off_listed);
    int64_t* n_items = reinterpret_cast<int64_t*>(base + l.off_nitems);
    int32_t* items = reinterpret_cast<int32_t*>(base + l.off_items);
    uint64_t* keys = reinterpret_cast<uint64_t*>(base + l.off_keys);
    int32_t* vals = reinterpret_cast<int32_t*>(base + l.off_vals);
    int32_t* sorted = reinterpret_cast<int32_t*>(base + l.off_sorted);
    hipError_t e;
    auto chk = [&]() { return (e = hipGetLastError()) == hipSuccess; };
    if (ext_status)
        p2p_copy_i32<<<1, kP2PThreads, 0, st>>>(ext_status, status);
    else
        p2p_set_i32<<<1, kP2PThreads, 0, st>>>(status, 0);
    if (!chk()) return e;
    if (check) {
        p2p_csr_check<<<p2p_grid(std::max<int64_t>((int64_t)n_leaves + 1, n_ulist)), kP2PThreads, 0, st>>>(
            src_ofs, trg_ofs, ulist_ofs, ulist, n_leaves, in.n_src, in.n_trg, n_ulist, status);
        if (!chk()) return e;
    }
    if (n_leaves > 0) {
        p2p_csr_count<<<p2p_grid(n_leaves), kP2PThreads, 0, st>>>(src_ofs, trg_ofs, ulist_ofs, ulist, n_leaves,
                                                                  status, cnt, listed);
        if (!chk()) return e;
        if ((e = exclusive_scan_i64(cnt, n_leaves, cnt, reinterpret_cast<int64_t*>(base + l.off_scan), n_items,
                                    st)) != hipSuccess)
            return e;
        p2p_item_slots<<<p2p_grid(l.max_items), kP2PThreads, 0, st>>>(l.max_items, keys, vals);
        if (!chk()) return e;
        p2p_csr_items<<<p2p_grid(n_leaves), kP2PThreads, 0, st>>>(trg_ofs, cnt, listed, n_leaves, l.max_items,
                                                                  items, keys);
        if (!chk()) return e;
        if ((e = radix_sort_pairs(keys, vals, l.max_items, kItemKeyBits, base + l.off_sort, l.sort, st)) !=
            hipSuccess)
            return e;
        p2p_item_order<<<p2p_grid(l.max_items), kP2PThreads, 0, st>>>(items, vals, n_items, sorted);
        if (!chk()) return e;
        const P2PItems it{src_ofs, trg_ofs, ulist_ofs, ulist, sorted, n_items, status, n_leaves, l.max_items};
        if ((e = run_p2p_any(in, it, out, accumulate, ws, st, timer)) != hipSuccess) return e;
    }
    p2p_poison<<<p2p_grid(3 * in.n_trg), kP2PThreads, 0, st>>>(status, out, 3 * in.n_trg);
    chk();
    return e;
}

// ---------------------------------------------------------------------------
// the layout check on its own, and the transposed lists (adjoint sums)
// ---------------------------------------------------------------------------
namespace {

__global__ __launch_bounds__(kP2PThreads) void p2p_t_init(int64_t nu, uint64_t* __restrict__ keys,
                                                          int32_t* __restrict__ vals) {
    for (int64_t k = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; k < nu; k += (int64_t)gridDim.x * kP2PThreads) {
        keys[k] = 0;
        vals[k] = 0;
    }
}

// entry k of leaf L's list: key = the listed leaf, value = L
__global__ __launch_bounds__(kP2PThreads) void p2p_t_keys(const int64_t* __restrict__ uo,
                                                          const int32_t* __restrict__ ul, int32_t nl,
                                                          const int32_t* __restrict__ status,
                                                          uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    if (*status != 0) return;                          // malformed: every entry stays at leaf 0
    for (int64_t L = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; L < nl; L += (int64_t)gridDim.x * kP2PThreads)
        for (int64_t k = uo[L]; k < uo[L + 1]; ++k) {
            keys[k] = (uint64_t)ul[k];
            vals[k] = (int32_t)L;
        }
}

// ofs[g] = first sorted position whose key is >= g, g in [0, nl]
__global__ __launch_bounds__(kP2PThreads) void p2p_t_offsets(const uint64_t* __restrict__ keys, int64_t n, int32_t nl,
                                                             int64_t* __restrict__ ofs) {
    for (int64_t i = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; i <= n; i += (int64_t)gridDim.x * kP2PThreads) {
        const int64_t kp = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t kc = i == n ? (int64_t)nl : (int64_t)keys[i];
        for (int64_t g = kp + 1; g <= kc; ++g) ofs[g] = i;
    }
}

int p2p_key_bits(int32_t nl) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < nl) ++b;
    return b;
}

struct TransposeLayout {
    SortLayout sort;
    size_t off_keys, off_sort, total;
};
TransposeLayout transpose_layout(int64_t nu) {
    TransposeLayout l{};
    l.sort = sort_layout(std::max<int64_t>(nu, 1));
    size_t off = 0;
    l.off_keys = off;
    off = align_up(off + (size_t)std::max<int64_t>(nu, 1) * 8, 256);
    l.off_sort = off;
    off = align_up(off + l.sort.total, 256);
    l.total = off;
    return l;
}

}  // namespace

hipError_t launch_p2p_check(int32_t n_leaves, const int64_t* src_ofs, const int64_t* trg_ofs,
                            const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_src, int64_t n_trg,
                            int64_t n_ulist, int32_t* status, hipStream_t st) {
    p2p_set_i32<<<1, kP2PThreads, 0, st>>>(status, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    p2p_csr_check<<<p2p_grid(std::max<int64_t>((int64_t)n_leaves + 1, n_ulist)), kP2PThreads, 0, st>>>(
        src_ofs, trg_ofs, ulist_ofs, ulist, n_leaves, n_src, n_trg, n_ulist, status);
    return hipGetLastError();
}

size_t p2p_transpose_bytes(int64_t n_ulist) { return transpose_layout(n_ulist).total; }

hipError_t launch_p2p_transpose(int32_t n_leaves, const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist,
                                const int32_t* status, int64_t* ulist_ofs_t, int32_t* ulist_t, void* ws,
                                hipStream_t st) {
    const TransposeLayout l = transpose_layout(n_ulist);
    uint64_t* keys = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + l.off_keys);
    hipError_t e;
    auto chk = [&]() { return (e = hipGetLastError()) == hipSuccess; };
    if (n_ulist > 0) {
        p2p_t_init<<<p2p_grid(n_ulist), kP2PThreads, 0, st>>>(n_ulist, keys, ulist_t);
        if (!chk()) return e;
        if (n_leaves > 0) {
            p2p_t_keys<<<p2p_grid(n_leaves), kP2PThreads, 0, st>>>(ulist_ofs, ulist, n_leaves, status, keys, ulist_t);
            if (!chk()) return e;
        }
        if ((e = radix_sort_pairs(keys, ulist_t, n_ulist, p2p_key_bits(n_leaves), static_cast<char*>(ws) + l.off_sort,
                                  l.sort, st)) != hipSuccess)
            return e;
    }
    p2p_t_offsets<<<p2p_grid(n_ulist + 1), kP2PThreads, 0, st>>>(keys, n_ulist, n_leaves, ulist_ofs_t);
    chk();
    return e;
}

// ---------------------------------------------------------------------------
// adjoints of the leaf-to-leaf sums (float64), with r_nm = x_n - y_m,
// q_m = w_m f_m (phi_m for the double layer), g_n = dL/du_n, c the forward's
// prefactor and the sums over n running over the targets of the leaves whose
// lists hold m's leaf (the transposed lists):
// single layer
//   dL/dx_n = c sum_m K(r_nm; g_n, q_m)          kernel 2, forward lists
//   dL/df_m = c w_m sum_n S(r_nm) g_n            kernel 0, transposed (S even in r)
//   dL/dy_m = c sum_n K(r_mn; q_m, g_n)          kernel 2, transposed (K odd in r,
//                                                symmetric in its two vectors)
// double layer
//   dL/dx_n   = c sum_m G(r_nm; n_m, q_m, g_n)   kernel 3, forward lists
//   dL/dphi_m = c w_m sum_n r (r.n_m)(r.g_n)/rho^5 with r = r_nm
//             = -c w_m sum_n r' (r'.n_m)(r'.g_n)/rho^5, r' = r_mn   kernel 4, transposed
//   dL/dy_m   = -c sum_n G(r_nm; ...) = -c sum_n G(r_mn; n_m, q_m, g_n)   kernel 5,
//               transposed (G even in r)
// ---------------------------------------------------------------------------
namespace {

struct P2PVjpLayout {
    size_t off_status, off_uot, off_ult, off_tws, off_q, off_tmp, off_p2p, total;
};

P2PVjpLayout p2p_vjp_layout(int kernel, int64_t ns, int64_t nt, int32_t nl, int64_t nu) {
    P2PVjpLayout l{};
    size_t off = 0;
    auto take = [&](size_t& o, size_t bytes) {
        o = off;
        off = align_up(off + std::max<size_t>(bytes, 8), 256);
    };
    take(l.off_status, sizeof(int32_t));
    take(l.off_uot, (size_t)(nl + 1) * 8);
    take(l.off_ult, (size_t)nu * 4);
    take(l.off_tws, p2p_transpose_bytes(nu));
    take(l.off_q, (size_t)ns * 24);
    take(l.off_tmp, (size_t)ns * 24);
    const int k_trg = kernel ? 3 : 2, k_f = kernel ? 4 : 0, k_src = kernel ? 5 : 2;
    const size_t p = std::max({p2p_workspace_bytes(k_trg, 0, ns, nt, nl), p2p_workspace_bytes(k_f, 0, nt, ns, nl),
                               p2p_workspace_bytes(k_src, 0, nt, ns, nl)});
    take(l.off_p2p, p);
    l.total = off;
    return l;
}

// q = w f, (3, n)
__global__ __launch_bounds__(kP2PThreads) void p2p_times_w(const double* __restrict__ w, const double* __restrict__ f,
                                                           int64_t n, double* __restrict__ q) {
    for (int64_t i = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kP2PThreads)
        for (int c = 0; c < 3; ++c) q[c * n + i] = w[i] * f[c * n + i];
}

// out (=|+=) w v, (3, n)
__global__ __launch_bounds__(kP2PThreads) void p2p_add_times_w(const double* __restrict__ w,
                                                               const double* __restrict__ v, int64_t n,
                                                               double* __restrict__ out, int accumulate) {
    for (int64_t i = (int64_t)blockIdx.x * kP2PThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kP2PThreads)
        for (int c = 0; c < 3; ++c) {
            const double val = w[i] * v[c * n + i];
            out[c * n + i] = accumulate ? out[c * n + i] + val : val;
        }
}

}  // namespace

size_t p2p_vjp_workspace_bytes(int kernel, int64_t n_src, int64_t n_trg, int32_t n_leaves, int64_t n_ulist) {
    if (n_src <= 0 || n_trg <= 0) return 0;
    return p2p_vjp_layout(kernel, n_src, n_trg, n_leaves, n_ulist).total;
}

hipError_t launch_p2p_vjp(const SumInputs& in, int32_t n_leaves, const int64_t* src_ofs, const int64_t* trg_ofs,
                          const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist, const double* grad_vel,
                          double* grad_density, double* grad_src, double* grad_trg, int accumulate, void* ws,
                          hipStream_t st) {
    const int64_t ns = in.n_src, nt = in.n_trg;
    const bool dl = in.kernel != 0;
    const P2PVjpLayout l = p2p_vjp_layout(in.kernel, ns, nt, n_leaves, n_ulist);
    char* base = static_cast<char*>(ws);
    int32_t* status = reinterpret_cast<int32_t*>(base + l.off_status);
    const KernelTimer none{};
    hipError_t e = launch_p2p_check(n_leaves, src_ofs, trg_ofs, ulist_ofs, ulist, ns, nt, n_ulist, status, st);
    if (e != hipSuccess) return e;
    if (grad_trg) {
        SumInputs t = in;
        t.kernel = dl ? 3 : 2;
        t.mixed = 0;
        t.trg_vec = grad_vel;
        t.pair_class = nullptr;
        e = launch_p2p_csr(t, n_leaves, src_ofs, trg_ofs, ulist_ofs, ulist, n_ulist, grad_trg, accumulate,
                           base + l.off_p2p, st, none, false, status);
        if (e != hipSuccess) return e;
    }
    if (!grad_density && !grad_src) return hipSuccess;
    int64_t* uot = reinterpret_cast<int64_t*>(base + l.off_uot);
    int32_t* ult = reinterpret_cast<int32_t*>(base + l.off_ult);
    if ((e = launch_p2p_transpose(n_leaves, ulist_ofs, ulist, n_ulist, status, uot, ult, base + l.off_tws, st)) !=
        hipSuccess)
        return e;
    // the transposed sums: the forward's sources are the targets, its targets
    // (carrying g, unit weights) the sources; the pair rule's groups swap; the
    // double layer's sums are odd in r there, hence -c
    SumInputs tr{};
    tr.n_src = nt;
    tr.src_xyz = in.trg_xyz;
    tr.density = grad_vel;
    tr.weight = nullptr;
    tr.n_trg = ns;
    tr.trg_xyz = in.src_xyz;
    tr.excl = in.excl;
    tr.src_group = in.trg_group;
    tr.trg_group = in.src_group;
    tr.pref = dl ? -in.pref : in.pref;
    if (grad_density) {
        double* tmp = reinterpret_cast<double*>(base + l.off_tmp);
        SumInputs f = tr;
        f.kernel = dl ? 4 : 0;
        f.trg_vec = dl ? in.normal : nullptr;
        e = launch_p2p_csr(f, n_leaves, trg_ofs, src_ofs, uot, ult, n_ulist, tmp, 0, base + l.off_p2p, st, none, false,
                           status);
        if (e != hipSuccess) return e;
        p2p_add_times_w<<<p2p_grid(ns), kP2PThreads, 0, st>>>(in.weight, tmp, ns, grad_density, accumulate);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (grad_src) {
        double* q = reinterpret_cast<double*>(base + l.off_q);
        p2p_times_w<<<p2p_grid(ns), kP2PThreads, 0, st>>>(in.weight, in.density, ns, q);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        SumInputs y = tr;
        y.kernel = dl ? 5 : 2;
        y.trg_vec = dl ? in.normal : q;
        y.trg_vec2 = dl ? q : nullptr;
        e = launch_p2p_csr(y, n_leaves, trg_ofs, src_ofs, uot, ult, n_ulist, grad_src, accumulate, base + l.off_p2p,
                           st, none, false, status);
    }
    return e;
}

// ---------------------------------------------------------------------------
// plan construction (host)
// ---------------------------------------------------------------------------
int p2p_plan_build(int device, int32_t n_leaves, int64_t n_src, int64_t n_trg,
                   const int64_t* src_ofs, const int64_t* trg_ofs, const int64_t* ulist_ofs,
                   const int32_t* ulist, int64_t n_ulist, stokes_p2p_plan** out, std::string& err) {
    auto check_ofs = [&](const int64_t* o, int64_t end, const char* name) -> bool {
        if (o[0] != 0) { err = std::string(name) + "[0] must be 0"; return false; }
        for (int32_t L = 0; L < n_leaves; ++L)
            if (o[L + 1] < o[L]) { err = std::string(name) + " must be non-decreasing"; return false; }
        if (o[n_leaves] != end) {
            err = std::string(name) + "[n_leaves] must equal " + std::to_string(end);
            return false;
        }
        return true;
    };
    if (!check_ofs(src_ofs, n_src, "src_leaf_ofs") || !check_ofs(trg_ofs, n_trg, "trg_leaf_ofs") ||
        !check_ofs(ulist_ofs, n_ulist, "ulist_ofs"))
        return STOKES_EINVAL;
    for (int64_t k = 0; k < n_ulist; ++k)
        if (ulist[k] < 0 || ulist[k] >= n_leaves) {
            err = "ulist entry " + std::to_string(k) + " is outside [0, n_leaves)";
            return STOKES_EINVAL;
        }
    // work items: (leaf, 64-target chunk), largest pair count first
    int64_t pairs = 0;
    struct Item { int64_t cost; int32_t leaf, chunk; };
    std::vector<Item> items;
    for (int32_t L = 0; L < n_leaves; ++L) {
        int64_t s = 0;
        for (int64_t k = ulist_ofs[L]; k < ulist_ofs[L + 1]; ++k) s += src_ofs[ulist[k] + 1] - src_ofs[ulist[k]];
        const int64_t nt = trg_ofs[L + 1] - trg_ofs[L];
        pairs += nt * s;
        for (int64_t c = 0; c * kWave < nt; ++c) {
            if (c > INT32_MAX) { err = "leaf too large"; return STOKES_EUNSUPPORTED; }
            // the pair loop of an n-target item runs s/R steps, R = min(16, 64/n)
            const int64_t n_c = std::min<int64_t>(kWave, nt - c * kWave);
            const int64_t rep = std::min<int64_t>(kMaxRep, kWave / n_c);
            items.push_back({s * 64 / rep + s + 1, L, (int32_t)c});
        }
    }
    if ((int64_t)items.size() > (int64_t)INT32_MAX) { err = "too many work items"; return STOKES_EUNSUPPORTED; }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<int32_t> flat(2 * items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        flat[2 * i] = items[i].leaf;
        flat[2 * i + 1] = items[i].chunk;
    }
    stokes_p2p_plan* p = new (std::nothrow) stokes_p2p_plan{};
    if (!p) { err = "out of host memory"; return STOKES_EDEVICE; }
    p->device = device;
    p->n_leaves = n_leaves;
    p->n_src = n_src;
    p->n_trg = n_trg;
    p->n_ulist = n_ulist;
    p->n_items = (int64_t)items.size();
    p->pairs = pairs;
    auto up = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
        return bytes == 0 || hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    const size_t ob = (size_t)(n_leaves + 1) * sizeof(int64_t);
    if (!up((void**)&p->d_src_ofs, src_ofs, ob) || !up((void**)&p->d_trg_ofs, trg_ofs, ob) ||
        !up((void**)&p->d_ulist_ofs, ulist_ofs, ob) ||
        !up((void**)&p->d_ulist, ulist, (size_t)n_ulist * sizeof(int32_t)) ||
        !up((void**)&p->d_items, flat.data(), flat.size() * sizeof(int32_t))) {
        p2p_plan_free(p);
        err = "device allocation or copy failed for the leaf layout";
        return STOKES_EDEVICE;
    }
    *out = p;
    return STOKES_OK;
}

void p2p_plan_free(stokes_p2p_plan* p) {
    if (!p) return;
    for (void* d : {(void*)p->d_src_ofs, (void*)p->d_trg_ofs, (void*)p->d_ulist_ofs, (void*)p->d_ulist,
                    (void*)p->d_items})
        if (d) (void)hipFree(d);
    delete p;
}

int64_t p2p_plan_info(const stokes_p2p_plan* p, int which) {
    switch (which) {
        case 0: return p->n_src;
        case 1: return p->n_trg;
        case 2: return p->n_leaves;
        case 3: return p->pairs;
        case 4: return p->device;
        default: return 0;
    }
}

}  // namespace stokes
