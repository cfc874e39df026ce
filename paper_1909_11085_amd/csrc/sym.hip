// Each-pair-once float64 single-layer sums over a shared point set: the
// forward sum and its adjoint.
//
// When the sources are the targets (one point array, one group array), the
// Stokeslet of eq. (sl_stokes) is symmetric, S(x, y) = S(y, x), and even in
// r = x - y, so one evaluation of the pair (i, j) serves both points:
//   * forward: q_j's velocity at x_i and q_i's velocity at x_j share the
//     offset, 1/rho and 1/rho^2; per unordered pair 10 shared float64
//     operations and 10 per direction, against 20 per ordered pair one-sided;
//   * adjoint of L(u) with g = dL/du: the density gradients S(r) g_j (at i)
//     and S(r) g_i (at j) share the offset and the dot products r.g, and the
//     position-gradient term V = K(r; g_i, q_j) + K(r; g_j, q_i) (K the
//     gradient in r of a.S(r)b) is odd in r, so x_i gains V and x_j loses V:
//     about 74 operations per unordered pair, against 55 per ordered pair.
//
// Design (gfx950, wave64):
//   * tiles of 64 points; a wave owns T consecutive tiles as rows (T points
//     per lane, in registers), a workgroup 4 T tiles (a row block);
//   * the triangle of (row block W, column tile b >= first tile of W) units
//     is cut into equal stream-K ranges, one per resident workgroup; rows
//     stay in registers along a range, their sums flushed as one segment per
//     (workgroup, row block);
//   * a unit: each lane takes one column point (its record and running sums)
//     and, 64 times, evaluates its T rows against it and passes the column
//     point with its sums on (within 16-lane rows by DPP, every 16 steps a
//     whole row on); after 64 steps every row of the wave has met every
//     column point and each column point is back in its lane with the
//     wave's sums;
//   * the 4 waves' column sums are added in LDS in a fixed order and stored
//     as the unit's column partial;
//   * units that may hold a pair needing a rule (a shared group id, or a
//     row point inside the column tile's box: possible zero distance) run the
//     same rotation with the masks (the column's group id rotates along);
//     a wave's own tiles run it too, the tile of the unit itself as the
//     diagonal: a lane takes the pair only when its point precedes the
//     column point, so every unordered pair of the tile counts once;
//   * the reduction adds, per point and in a fixed order, its row segments
//     and the column partials of its tile from every row block:
//     deterministic, no atomics.
// Positions are stored doubled (exact) as in the one-sided kernels; the
// factors this leaves are taken out in the reduction.
#include <algorithm>

#include "direct_dev.hpp"

// rows per lane (T) and minimum waves per SIMD (W): forward and adjoint
#ifndef STOKES_SYM_T64
#define STOKES_SYM_T64 6
#endif
#ifndef STOKES_SYM_W64
#define STOKES_SYM_W64 2
#endif
#ifndef STOKES_SYM_TV
#define STOKES_SYM_TV 4
#endif
#ifndef STOKES_SYM_WV
#define STOKES_SYM_WV 2
#endif

namespace stokes {

namespace {

// Point record: doubled position and six doubles (forward: q and 4q;
// adjoint: q and g), the layout of the one-sided single-layer record.
struct alignas(16) SymRec { double x, y, z, d[6], pad; };
static_assert(sizeof(SymRec) == sizeof(SrcSL64x), "the prep kernel writes this layout");

struct SymArgs {
    SumInputs in;
    const SymRec* rec;        // n_pad records
    const int32_t* grp;       // n_pad group ids
    const SubMeta* meta;      // per 64-point tile
    int64_t n_pad, NT, NW, units;
    double* row_part;         // (grid + NW) segments of NA x (kBlock T) doubles
    double* col_part;         // (units, NA, 64)
    double* out0;             // forward: velocity; adjoint: dL/df (either may be null in the adjoint)
    double* out1;             // adjoint: dL/dx, the total position gradient
    int accumulate;
};

// units of the row blocks before W (row block W holds NT - tpb W units)
__host__ __device__ __forceinline__ int64_t sym_off(int64_t W, int64_t NT, int64_t tpb) {
    return W * NT - tpb * (W * (W - 1) / 2);
}

// the row block holding unit u: largest W with sym_off(W) <= u
__device__ __forceinline__ int64_t sym_block_of(int64_t u, int64_t NT, int64_t tpb, int64_t NW) {
    int64_t lo = 0, hi = NW - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (sym_off(mid, NT, tpb) <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The column points move through the wave in 4 phases: within each row of 16
// lanes, lane i takes lane i-1's value (DPP row_ror:1) 16 times, then every
// lane takes the value of the lane 16 below it (whole rows one row on,
// through the LDS crossbar).  After the 4 phases every lane has held each of
// the 64 column points once and each is back in its own lane.
__device__ __forceinline__ int row_rot(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x121, 0xF, 0xF, true); }
__device__ __forceinline__ double row_rot(double v) {
    return __hiloint2double(row_rot(__double2hiint(v)), row_rot(__double2loint(v)));
}
__device__ __forceinline__ int cross_rot(int v, int addr) { return __builtin_amdgcn_ds_bpermute(addr, v); }
__device__ __forceinline__ double cross_rot(double v, int addr) {
    return __hiloint2double(cross_rot(__double2hiint(v), addr), cross_rot(__double2loint(v), addr));
}
// byte address for cross_rot: the lane 16 below, cyclically
__device__ __forceinline__ int cross_addr(int lane) { return ((lane - 16) & (kWave - 1)) * 4; }
// the column point (0..63 in its tile) that lane holds in phase R at step sp
__device__ __forceinline__ int held_col(int lane, int R, int sp) {
    return ((((lane >> 4) - R) & 3) << 4) | (((lane & 15) - sp) & 15);
}

// ---------------------------------------------------------------------------
// pair functions (D = 2r from doubled positions; ri = 1/rho; MASKED: nothing
// for skip or zero distance, 1/rho taken as 0)
// ---------------------------------------------------------------------------

// Forward: record d = (q, 4q).  The row gains 4[q_c/rho + r (r.q_c)/rho^3],
// the column 4[q_r/rho + r (r.q_r)/rho^3] (S is even in r).
struct FwdSL {
    static constexpr int NA = 3;
    template <bool MASKED>
    __device__ __forceinline__ static void pair(double x, double y, double z, const double (&r)[6],
                                                double (&ra)[NA], double cx, double cy, double cz,
                                                const double (&c)[6], double (&ca)[NA], bool skip) {
        const double dx = x - cx, dy = y - cy, dz = z - cz;
        const double A = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        const double ri = rinv_doubled(A, MASKED && (skip || A == 0.0));
        const double ri2 = ri * ri;
        const double rc = __builtin_fma(dx, c[0], __builtin_fma(dy, c[1], dz * c[2])) * ri2;
        ra[0] = __builtin_fma(__builtin_fma(rc, dx, c[3]), ri, ra[0]);
        ra[1] = __builtin_fma(__builtin_fma(rc, dy, c[4]), ri, ra[1]);
        ra[2] = __builtin_fma(__builtin_fma(rc, dz, c[5]), ri, ra[2]);
        const double rr = __builtin_fma(dx, r[0], __builtin_fma(dy, r[1], dz * r[2])) * ri2;
        ca[0] = __builtin_fma(__builtin_fma(rr, dx, r[3]), ri, ca[0]);
        ca[1] = __builtin_fma(__builtin_fma(rr, dy, r[4]), ri, ca[1]);
        ca[2] = __builtin_fma(__builtin_fma(rr, dz, r[5]), ri, ca[2]);
    }
};

// Adjoint: record d = (q, g).  Accumulators 0..2: the sum of S(r) g over the
// other point (dL/df before c w), 3..5: twice the sum of +-V, with
//   V = K(r; g_r, q_c) + K(r; g_c, q_r)
//     = [(r.q_c) g_r + (r.g_r) q_c + (r.q_r) g_c + (r.g_c) q_r - C r]/rho^3
//       - 3 [(r.g_r)(r.q_c) + (r.g_c)(r.q_r)] r/rho^5,   C = g_r.q_c + g_c.q_r,
// the row's r = x_r - x_c; the row gains V, the column -V (K is odd in r).
// With D = 2r the dot products are doubled; the bracket is formed as
//   [P - (C + 3/4 (a1 b1 + a2 b2)/rho^2) D] / rho^3 = 2 V,
// P = b1 g_r + a1 q_c + b2 g_c + a2 q_r, a1 = D.g_r, b1 = D.q_c, a2 = D.g_c,
// b2 = D.q_r, and S(r) g_c = [g_c + (a2/4)/rho^2 D]/rho.
struct VjpSL {
    static constexpr int NA = 6;
    template <bool MASKED>
    __device__ __forceinline__ static void pair(double x, double y, double z, const double (&r)[6],
                                                double (&ra)[NA], double cx, double cy, double cz,
                                                const double (&c)[6], double (&ca)[NA], bool skip) {
        const double dx = x - cx, dy = y - cy, dz = z - cz;
        const double A = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
        const double ri = rinv_doubled(A, MASKED && (skip || A == 0.0));
        const double ri2 = ri * ri;
        const double ri3 = ri2 * ri;
        const double ri2q = 0.25 * ri2;
        const double a1 = __builtin_fma(dx, r[3], __builtin_fma(dy, r[4], dz * r[5]));   // D.g_r
        const double b1 = __builtin_fma(dx, c[0], __builtin_fma(dy, c[1], dz * c[2]));   // D.q_c
        const double a2 = __builtin_fma(dx, c[3], __builtin_fma(dy, c[4], dz * c[5]));   // D.g_c
        const double b2 = __builtin_fma(dx, r[0], __builtin_fma(dy, r[1], dz * r[2]));   // D.q_r
        const double C = __builtin_fma(r[3], c[0], __builtin_fma(r[4], c[1], __builtin_fma(r[5], c[2],
                         __builtin_fma(c[3], r[0], __builtin_fma(c[4], r[1], c[5] * r[2])))));
        const double k = __builtin_fma(0.75 * __builtin_fma(a1, b1, a2 * b2), ri2, C);
        const double px = __builtin_fma(b1, r[3], __builtin_fma(a1, c[0], __builtin_fma(b2, c[3], a2 * r[0])));
        const double py = __builtin_fma(b1, r[4], __builtin_fma(a1, c[1], __builtin_fma(b2, c[4], a2 * r[1])));
        const double pz = __builtin_fma(b1, r[5], __builtin_fma(a1, c[2], __builtin_fma(b2, c[5], a2 * r[2])));
        const double vx = __builtin_fma(-k, dx, px) * ri3;
        const double vy = __builtin_fma(-k, dy, py) * ri3;
        const double vz = __builtin_fma(-k, dz, pz) * ri3;
        ra[3] += vx; ra[4] += vy; ra[5] += vz;
        ca[3] -= vx; ca[4] -= vy; ca[5] -= vz;
        const double sr = a2 * ri2q, sc = a1 * ri2q;
        ra[0] = __builtin_fma(__builtin_fma(sr, dx, c[3]), ri, ra[0]);
        ra[1] = __builtin_fma(__builtin_fma(sr, dy, c[4]), ri, ra[1]);
        ra[2] = __builtin_fma(__builtin_fma(sr, dz, c[5]), ri, ra[2]);
        ca[0] = __builtin_fma(__builtin_fma(sc, dx, r[3]), ri, ca[0]);
        ca[1] = __builtin_fma(__builtin_fma(sc, dy, r[4]), ri, ca[1]);
        ca[2] = __builtin_fma(__builtin_fma(sc, dz, r[5]), ri, ca[2]);
    }
};

template <int NA, int T>
__device__ __forceinline__ void flush_sym_segment(const SymArgs& a, int64_t W, int wave, int lane,
                                                  const double (&ra)[T][NA]) {
    constexpr int RB = kBlock * T;
    double* seg = a.row_part + (int64_t)(blockIdx.x + W) * NA * RB;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int li = wave * (kWave * T) + k * kWave + lane;
#pragma unroll
        for (int j = 0; j < NA; ++j) seg[j * RB + li] = ra[k][j];
    }
}

template <int NA>
__device__ __forceinline__ void rotate_col_row(double& cx, double& cy, double& cz, double (&cd)[6],
                                               double (&ca)[NA]) {
    cx = row_rot(cx); cy = row_rot(cy); cz = row_rot(cz);
#pragma unroll
    for (int j = 0; j < 6; ++j) cd[j] = row_rot(cd[j]);
#pragma unroll
    for (int j = 0; j < NA; ++j) ca[j] = row_rot(ca[j]);
}
template <int NA>
__device__ __forceinline__ void rotate_col_cross(double& cx, double& cy, double& cz, double (&cd)[6],
                                                 double (&ca)[NA], int xa) {
    cx = cross_rot(cx, xa); cy = cross_rot(cy, xa); cz = cross_rot(cz, xa);
#pragma unroll
    for (int j = 0; j < 6; ++j) cd[j] = cross_rot(cd[j], xa);
#pragma unroll
    for (int j = 0; j < NA; ++j) ca[j] = cross_rot(ca[j], xa);
}

template <class P, int T, int W_SIMD>
__global__ __launch_bounds__(kBlock, W_SIMD) void sym_main(SymArgs a) {
    constexpr int NA = P::NA;
    constexpr int TPB = 4 * T;
    __shared__ double s_col[4][NA][kWave];
    const int64_t U = a.units, G = gridDim.x, NT = a.NT;
    const int64_t u0 = unit_begin(blockIdx.x, U, G), u1 = unit_begin(blockIdx.x + 1, U, G);
    if (u0 >= u1) return;                      // whole workgroup idle (uniform)
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const bool excl = a.in.excl != 0;
    const SymRec* rec = a.rec;

    Targets<T> t;
    Box wbox{};
    double rd[T][6], ra[T][NA];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int j = 0; j < NA; ++j) ra[k][j] = 0.0;
    bool wave_active = false;
    int64_t W = sym_block_of(u0, NT, TPB, a.NW);
    int64_t b = u0 - sym_off(W, NT, TPB) + TPB * W;
    int64_t Wcur = -1;
    for (int64_t u = u0; u < u1; ++u) {
        if (W != Wcur) {
            if (Wcur >= 0) flush_sym_segment<NA, T>(a, Wcur, wave, lane, ra);
            Wcur = W;
            const int64_t p0 = (TPB * W + T * wave) * kWave;
            wave_active = p0 < a.in.n_trg;
            wbox = load_targets<T>(a.in, wave_active ? p0 : 0, lane, t);
            double_targets<T>(t, &wbox);
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const SymRec r = rec[p0 + k * kWave + lane];   // p0 + T*64 <= n_pad
#pragma unroll
                for (int j = 0; j < 6; ++j) rd[k][j] = r.d[j];
#pragma unroll
                for (int j = 0; j < NA; ++j) ra[k][j] = 0.0;
            }
        }
        const int64_t A = TPB * W + T * wave;    // the wave's first tile
        // slots meeting every column point (full) and the slot whose tile is
        // b (diag: each unordered pair of the tile once); masked when a pair
        // may need the group or zero-distance rule
        uint32_t full = 0, diag = 0;
        bool masked = false;
        if (wave_active && b >= A) {
            const SubMeta m = a.meta[b];
            if (m.count > 0) {
                if (b >= A + T) {
                    full = (1u << T) - 1u;
                    masked = needs_near<T, false>(wbox, t, m, excl);
                } else {
                    const int d = (int)(b - A);
                    full = (1u << d) - 1u;
                    diag = 1u << d;
                    masked = true;
                }
            }
        }
        double ca[NA];
#pragma unroll
        for (int j = 0; j < NA; ++j) ca[j] = 0.0;
        if (full | diag) {
            const SymRec c = rec[b * kWave + lane];
            double cx = c.x, cy = c.y, cz = c.z, cd[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) cd[j] = c.d[j];
            const int xa = cross_addr(lane);
            if (!masked) {
                for (int R = 0; R < 4; ++R) {
#pragma unroll 1
                    for (int sp = 0; sp < 16; ++sp) {
#pragma unroll
                        for (int k = 0; k < T; ++k)
                            P::template pair<false>(t.x[k], t.y[k], t.z[k], rd[k], ra[k], cx, cy, cz, cd, ca, false);
                        rotate_col_row<NA>(cx, cy, cz, cd, ca);
                    }
                    rotate_col_cross<NA>(cx, cy, cz, cd, ca, xa);
                }
            } else {
                int cg = a.grp[b * kWave + lane];
                const uint32_t any = full | diag;
                for (int R = 0; R < 4; ++R) {
#pragma unroll 1
                    for (int sp = 0; sp < 16; ++sp) {
                        // the diagonal slot takes each unordered pair of its tile
                        // once: when this lane's point precedes the column point
                        const bool dpair = lane < held_col(lane, R, sp);
#pragma unroll
                        for (int k = 0; k < T; ++k) {
                            if (!((any >> k) & 1u)) continue;
                            const bool on = ((full >> k) & 1u) || dpair;
                            P::template pair<true>(t.x[k], t.y[k], t.z[k], rd[k], ra[k], cx, cy, cz, cd, ca,
                                                   !on || (excl && t.g[k] == cg));
                        }
                        rotate_col_row<NA>(cx, cy, cz, cd, ca);
                        cg = row_rot(cg);
                    }
                    rotate_col_cross<NA>(cx, cy, cz, cd, ca, xa);
                    cg = cross_rot(cg, xa);
                }
            }
        }
        __syncthreads();                       // the previous unit's sums have been read
#pragma unroll
        for (int j = 0; j < NA; ++j) s_col[wave][j][lane] = ca[j];
        __syncthreads();
        for (int i = threadIdx.x; i < NA * kWave; i += kBlock) {
            const int j = i >> 6, l = i & (kWave - 1);
            a.col_part[u * NA * kWave + i] = ((s_col[0][j][l] + s_col[1][j][l]) + s_col[2][j][l]) + s_col[3][j][l];
        }
        if (++b == NT) {
            ++W;
            b = TPB * W;
        }
    }
    flush_sym_segment<NA, T>(a, Wcur, wave, lane, ra);
}

__device__ __forceinline__ void put(double* out, int64_t o, double v, int accumulate) {
    out[o] = accumulate ? out[o] + v : v;
}

// out (=|+=) the prefactored sums of each point: its row segments and the
// column partials of its tile from every row block, in a fixed order.
template <class P, int T>
__global__ __launch_bounds__(kBlock) void sym_reduce(SymArgs a, int64_t grid) {
    constexpr int NA = P::NA;
    constexpr int TPB = 4 * T, RB = kBlock * T;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n = a.in.n_trg;
    if (p >= n) return;
    const int64_t NT = a.NT, U = a.units;
    const int64_t W = p / RB, li = p % RB, b = p / kWave, l = p % kWave;
    const int64_t g0 = unit_owner(sym_off(W, NT, TPB), U, grid);
    const int64_t g1 = unit_owner(sym_off(W + 1, NT, TPB) - 1, U, grid);
    double s[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) s[j] = 0.0;
    for (int64_t g = g0; g <= g1; ++g) {
        const double* seg = a.row_part + (g + W) * NA * RB;
#pragma unroll
        for (int j = 0; j < NA; ++j) s[j] += seg[j * RB + li];
    }
    for (int64_t Wp = 0; Wp * TPB <= b; ++Wp) {
        const double* cp = a.col_part + (sym_off(Wp, NT, TPB) + b - TPB * Wp) * NA * kWave;
#pragma unroll
        for (int j = 0; j < NA; ++j) s[j] += cp[j * kWave + l];
    }
    if constexpr (NA == 3) {
        // forward: 4 times the bare sums (doubled positions)
#pragma unroll
        for (int c = 0; c < 3; ++c) put(a.out0, c * n + p, 0.25 * a.in.pref * s[c], a.accumulate);
    } else {
        // adjoint: dL/df = c w sum S(r) g; dL/dx = c sum (+-V), accumulated as 2 V
        const double cw = a.in.pref * a.in.weight[p];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (a.out0) put(a.out0, c * n + p, cw * s[c], a.accumulate);
            if (a.out1) put(a.out1, c * n + p, 0.5 * a.in.pref * s[3 + c], a.accumulate);
        }
    }
}

// adjoint records: d[3..5] = g = dL/du at the point (zero for padding)
__global__ __launch_bounds__(kBlock) void sym_vjp_set_g(SymRec* rec, const double* g, int64_t n, int64_t n_pad) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_pad) return;
    const bool v = i < n;
    rec[i].d[3] = v ? g[i] : 0.0;
    rec[i].d[4] = v ? g[n + i] : 0.0;
    rec[i].d[5] = v ? g[2 * n + i] : 0.0;
}

constexpr int kSymT64 = STOKES_SYM_T64;
constexpr int kSymTV = STOKES_SYM_TV;

}  // namespace

int sym_blocks_per_cu(int adjoint) {
    int nb = 0;
    const hipError_t e =
        adjoint ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sym_main<VjpSL, kSymTV, STOKES_SYM_WV>, kBlock, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sym_main<FwdSL, kSymT64, STOKES_SYM_W64>,
                                                               kBlock, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

SymPlan plan_sym(int adjoint, int64_t n, int resident_blocks, int forced_grid) {
    SymPlan p{};
    p.T = adjoint ? kSymTV : kSymT64;
    const int na = adjoint ? VjpSL::NA : FwdSL::NA;
    const int64_t rb = (int64_t)kBlock * p.T;
    const int64_t tpb = 4 * (int64_t)p.T;
    p.n_pad = ceil_div(n, rb) * rb;
    p.NT = p.n_pad / kWave;
    p.NW = p.n_pad / rb;
    p.units = sym_off(p.NW, p.NT, tpb);
    const int64_t g = forced_grid > 0 ? forced_grid : std::max(1, resident_blocks);
    p.grid = std::max<int64_t>(1, std::min<int64_t>(g, p.units));
    size_t off = 0;
    p.off_rec = off;
    off = align_up(off + (size_t)p.n_pad * sizeof(SymRec), 256);
    p.off_aux = off;
    off = align_up(off + (size_t)p.n_pad * sizeof(int32_t), 256);
    p.off_meta = off;
    off = align_up(off + (size_t)p.NT * sizeof(SubMeta), 256);
    p.off_row = off;
    off = align_up(off + (size_t)(p.grid + p.NW) * na * (size_t)rb * sizeof(double), 256);
    p.off_col = off;
    off = align_up(off + (size_t)p.units * na * kWave * sizeof(double), 256);
    p.total = off;
    return p;
}

static SymArgs sym_args(const SumInputs& in, const SymPlan& p, void* ws) {
    char* base = static_cast<char*>(ws);
    SymArgs a{};
    a.in = in;
    a.rec = reinterpret_cast<const SymRec*>(base + p.off_rec);
    a.grp = reinterpret_cast<const int32_t*>(base + p.off_aux);
    a.meta = reinterpret_cast<const SubMeta*>(base + p.off_meta);
    a.n_pad = p.n_pad;
    a.NT = p.NT;
    a.NW = p.NW;
    a.units = p.units;
    a.row_part = reinterpret_cast<double*>(base + p.off_row);
    a.col_part = reinterpret_cast<double*>(base + p.off_col);
    return a;
}

hipError_t launch_sym(const SumInputs& in, const SymPlan& p, double* out, int accumulate, void* ws,
                      hipStream_t stream, const KernelTimer& timer) {
    if (in.n_trg <= 0) return hipSuccess;
    if (in.kernel != 0 || in.mixed) return hipErrorNotSupported;
    SymArgs a = sym_args(in, p, ws);
    a.out0 = out;
    a.accumulate = accumulate;
    char* base = static_cast<char*>(ws);
    hipError_t e = launch_prep(in, p.n_pad, base + p.off_rec, base + p.off_aux,
                               reinterpret_cast<SubMeta*>(base + p.off_meta), stream);
    if (e != hipSuccess) return e;
    if (timer.on()) (void)hipEventRecord(timer.start, stream);
    sym_main<FwdSL, kSymT64, STOKES_SYM_W64><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (timer.on()) (void)hipEventRecord(timer.stop, stream);
    if (e != hipSuccess) return e;
    sym_reduce<FwdSL, kSymT64><<<dim3((unsigned)ceil_div(in.n_trg, kBlock)), dim3(kBlock), 0, stream>>>(a, p.grid);
    return hipGetLastError();
}

hipError_t launch_sym_vjp(const SumInputs& in, const SymPlan& p, const double* grad_vel, double* grad_density,
                          double* grad_xyz, int accumulate, void* ws, hipStream_t stream,
                          const KernelTimer& timer) {
    if (in.n_trg <= 0) return hipSuccess;
    SymArgs a = sym_args(in, p, ws);
    a.out0 = grad_density;
    a.out1 = grad_xyz;
    a.accumulate = accumulate;
    char* base = static_cast<char*>(ws);
    SumInputs pin = in;                        // records: doubled position, q, then g in place of 4q
    pin.kernel = 0;
    pin.mixed = 0;
    hipError_t e = launch_prep(pin, p.n_pad, base + p.off_rec, base + p.off_aux,
                               reinterpret_cast<SubMeta*>(base + p.off_meta), stream);
    if (e != hipSuccess) return e;
    sym_vjp_set_g<<<dim3((unsigned)(p.n_pad / kBlock)), dim3(kBlock), 0, stream>>>(
        reinterpret_cast<SymRec*>(base + p.off_rec), grad_vel, in.n_trg, p.n_pad);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (timer.on()) (void)hipEventRecord(timer.start, stream);
    sym_main<VjpSL, kSymTV, STOKES_SYM_WV><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (timer.on()) (void)hipEventRecord(timer.stop, stream);
    if (e != hipSuccess) return e;
    sym_reduce<VjpSL, kSymTV><<<dim3((unsigned)ceil_div(in.n_trg, kBlock)), dim3(kBlock), 0, stream>>>(a, p.grid);
    return hipGetLastError();
}

}  // namespace stokes
