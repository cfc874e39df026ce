// Each-pair-once single-layer sum over a shared point set.
//
// When the sources are the targets (one point array, one group array), the
// Stokeslet of eq. (sl_stokes) is symmetric, S(x, y) = S(y, x), and even in
// r = x - y, so the pair (i, j) gives q_j's velocity at x_i and q_i's velocity
// at x_j from one offset, one 1/rho and one 1/rho^2.  Per unordered pair this
// is 10 shared float64 operations (offset, rho^2, 1/rho with one Newton step,
// 1/rho^2) and 10 per direction (r.q, its scale, three fused multiply-adds of
// q/rho + r (r.q)/rho^3), against 20 per ordered pair one-sided.
//
// Design (gfx950, wave64):
//   * tiles of 64 points; a wave owns T consecutive tiles as rows (T points
//     per lane, in registers), a workgroup 4 T tiles (a row block);
//   * the triangle of (row block W, column tile b >= first tile of W) units
//     is cut into equal stream-K ranges, one per resident workgroup; rows
//     stay in registers along a range, their sums flushed as one segment per
//     (workgroup, row block);
//   * a unit: each lane takes one column point (position, q, 4q and its
//     running sum) and, 64 times, evaluates its T rows against it and passes
//     the column point with its sum on (within 16-lane rows by DPP, every 16
//     steps a whole row on); after 64 steps every row of the wave has met
//     every column point and each column point is back in its lane with the
//     wave's sum;
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
// Positions are stored doubled (exact) as in the one-sided kernels, so the
// float64 sums are 4 times the bare ones.
#include <algorithm>

#include "direct_dev.hpp"

#ifndef STOKES_SYM_T64
#define STOKES_SYM_T64 6
#endif
#ifndef STOKES_SYM_W64
#define STOKES_SYM_W64 2
#endif

namespace stokes {

namespace {

constexpr int kSymT64 = STOKES_SYM_T64;
constexpr int kColVals = 3 * kWave;       // doubles of one unit's column partial

struct SymArgs {
    SumInputs in;
    const void* rec;          // packed records, n_pad
    const void* aux;          // int32 groups
    const SubMeta* meta;      // per 64-point tile
    int64_t n_pad, NT, NW, units;
    double* row_part;         // (grid + NW) segments of 3 x (kBlock T) doubles
    double* col_part;         // (units, 3, 64)
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
// the 64 column points once and each is back in its own lane.  (A rotation
// across the whole wave in one DPP step, wave_ror, costs several times a
// row rotation on this hardware.)
__device__ __forceinline__ int row_rot(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x121, 0xF, 0xF, true); }
__device__ __forceinline__ float row_rot(float v) { return __int_as_float(row_rot(__float_as_int(v))); }
__device__ __forceinline__ double row_rot(double v) {
    return __hiloint2double(row_rot(__double2hiint(v)), row_rot(__double2loint(v)));
}
__device__ __forceinline__ int cross_rot(int v, int addr) { return __builtin_amdgcn_ds_bpermute(addr, v); }
__device__ __forceinline__ float cross_rot(float v, int addr) { return __int_as_float(cross_rot(__float_as_int(v), addr)); }
__device__ __forceinline__ double cross_rot(double v, int addr) {
    return __hiloint2double(cross_rot(__double2hiint(v), addr), cross_rot(__double2loint(v), addr));
}
// byte address for cross_rot: the lane 16 below, cyclically
__device__ __forceinline__ int cross_addr(int lane) { return ((lane - 16) & (kWave - 1)) * 4; }
// the column point (0..63 in its tile) that lane holds in phase R at step sp
__device__ __forceinline__ int held_col(int lane, int R, int sp) {
    return ((((lane >> 4) - R) & 3) << 4) | (((lane & 15) - sp) & 15);
}

// One unordered pair, both directions, float64 on doubled positions:
// D = 2r, ri = 1/rho; the row gains 4[q_c/rho + r (r.q_c)/rho^3], the column
// 4[q_r/rho + r (r.q_r)/rho^3] (S is even in r).  MASKED: nothing for skip
// or zero distance (1/rho taken as 0).
template <bool MASKED>
__device__ __forceinline__ void pair_sym_f64(double x, double y, double z, double qx, double qy, double qz,
                                             double px, double py, double pz, double cx, double cy,
                                             double cz, double cqx, double cqy, double cqz, double cpx,
                                             double cpy, double cpz, bool skip, double& ax, double& ay,
                                             double& az, double& bx, double& by, double& bz) {
    const double dx = x - cx, dy = y - cy, dz = z - cz;
    const double A = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double ri = rinv_doubled(A, MASKED && (skip || A == 0.0));
    const double ri2 = ri * ri;
    const double rc = __builtin_fma(dx, cqx, __builtin_fma(dy, cqy, dz * cqz)) * ri2;
    ax = __builtin_fma(__builtin_fma(rc, dx, cpx), ri, ax);
    ay = __builtin_fma(__builtin_fma(rc, dy, cpy), ri, ay);
    az = __builtin_fma(__builtin_fma(rc, dz, cpz), ri, az);
    const double rr = __builtin_fma(dx, qx, __builtin_fma(dy, qy, dz * qz)) * ri2;
    bx = __builtin_fma(__builtin_fma(rr, dx, px), ri, bx);
    by = __builtin_fma(__builtin_fma(rr, dy, py), ri, by);
    bz = __builtin_fma(__builtin_fma(rr, dz, pz), ri, bz);
}

template <int T>
__device__ __forceinline__ void flush_sym_segment(const SymArgs& a, int64_t W, int wave, int lane,
                                                  const double (&ax)[T], const double (&ay)[T],
                                                  const double (&az)[T]) {
    constexpr int RB = kBlock * T;
    double* seg = a.row_part + (int64_t)(blockIdx.x + W) * 3 * RB;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int li = wave * (kWave * T) + k * kWave + lane;
        seg[li] = ax[k];
        seg[RB + li] = ay[k];
        seg[2 * RB + li] = az[k];
    }
}

template <int T>
__global__ __launch_bounds__(kBlock, STOKES_SYM_W64) void sym_main_f64(SymArgs a) {
    using Rec = SrcSL64x;
    constexpr int TPB = 4 * T;
    __shared__ double s_col[4][3][kWave];
    const int64_t U = a.units, G = gridDim.x, NT = a.NT;
    const int64_t u0 = unit_begin(blockIdx.x, U, G), u1 = unit_begin(blockIdx.x + 1, U, G);
    if (u0 >= u1) return;                      // whole workgroup idle (uniform)
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const bool excl = a.in.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    const int32_t* grp = reinterpret_cast<const int32_t*>(a.aux);

    Targets<T> t;
    Box wbox{};
    double qx[T], qy[T], qz[T], px[T], py[T], pz[T], ax[T], ay[T], az[T];
#pragma unroll
    for (int k = 0; k < T; ++k) ax[k] = ay[k] = az[k] = 0.0;
    bool wave_active = false;
    int64_t W = sym_block_of(u0, NT, TPB, a.NW);
    int64_t b = u0 - sym_off(W, NT, TPB) + TPB * W;
    int64_t Wcur = -1;
    for (int64_t u = u0; u < u1; ++u) {
        if (W != Wcur) {
            if (Wcur >= 0) flush_sym_segment<T>(a, Wcur, wave, lane, ax, ay, az);
            Wcur = W;
            const int64_t p0 = (TPB * W + T * wave) * kWave;
            wave_active = p0 < a.in.n_trg;
            wbox = load_targets<T>(a.in, wave_active ? p0 : 0, lane, t);
            double_targets<T>(t, &wbox);
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const Rec r = rec[p0 + k * kWave + lane];   // p0 + T*64 <= n_pad
                qx[k] = r.qx; qy[k] = r.qy; qz[k] = r.qz;
                px[k] = r.q4x; py[k] = r.q4y; pz[k] = r.q4z;
                ax[k] = ay[k] = az[k] = 0.0;
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
        double bx = 0.0, by = 0.0, bz = 0.0;
        if (full | diag) {
            const Rec c = rec[b * kWave + lane];
            double cx = c.x, cy = c.y, cz = c.z, cqx = c.qx, cqy = c.qy, cqz = c.qz;
            double cpx = c.q4x, cpy = c.q4y, cpz = c.q4z;
            const int xa = cross_addr(lane);
            if (!masked) {
                for (int R = 0; R < 4; ++R) {
#pragma unroll 1
                    for (int sp = 0; sp < 16; ++sp) {
#pragma unroll
                        for (int k = 0; k < T; ++k)
                            pair_sym_f64<false>(t.x[k], t.y[k], t.z[k], qx[k], qy[k], qz[k], px[k], py[k], pz[k],
                                                cx, cy, cz, cqx, cqy, cqz, cpx, cpy, cpz, false, ax[k], ay[k], az[k],
                                                bx, by, bz);
                        cx = row_rot(cx); cy = row_rot(cy); cz = row_rot(cz);
                        cqx = row_rot(cqx); cqy = row_rot(cqy); cqz = row_rot(cqz);
                        cpx = row_rot(cpx); cpy = row_rot(cpy); cpz = row_rot(cpz);
                        bx = row_rot(bx); by = row_rot(by); bz = row_rot(bz);
                    }
                    cx = cross_rot(cx, xa); cy = cross_rot(cy, xa); cz = cross_rot(cz, xa);
                    cqx = cross_rot(cqx, xa); cqy = cross_rot(cqy, xa); cqz = cross_rot(cqz, xa);
                    cpx = cross_rot(cpx, xa); cpy = cross_rot(cpy, xa); cpz = cross_rot(cpz, xa);
                    bx = cross_rot(bx, xa); by = cross_rot(by, xa); bz = cross_rot(bz, xa);
                }
            } else {
                int cg = grp[b * kWave + lane];
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
                            pair_sym_f64<true>(t.x[k], t.y[k], t.z[k], qx[k], qy[k], qz[k], px[k], py[k], pz[k],
                                               cx, cy, cz, cqx, cqy, cqz, cpx, cpy, cpz,
                                               !on || (excl && t.g[k] == cg), ax[k], ay[k], az[k], bx, by, bz);
                        }
                        cx = row_rot(cx); cy = row_rot(cy); cz = row_rot(cz);
                        cqx = row_rot(cqx); cqy = row_rot(cqy); cqz = row_rot(cqz);
                        cpx = row_rot(cpx); cpy = row_rot(cpy); cpz = row_rot(cpz);
                        bx = row_rot(bx); by = row_rot(by); bz = row_rot(bz);
                        cg = row_rot(cg);
                    }
                    cx = cross_rot(cx, xa); cy = cross_rot(cy, xa); cz = cross_rot(cz, xa);
                    cqx = cross_rot(cqx, xa); cqy = cross_rot(cqy, xa); cqz = cross_rot(cqz, xa);
                    cpx = cross_rot(cpx, xa); cpy = cross_rot(cpy, xa); cpz = cross_rot(cpz, xa);
                    bx = cross_rot(bx, xa); by = cross_rot(by, xa); bz = cross_rot(bz, xa);
                    cg = cross_rot(cg, xa);
                }
            }
        }
        __syncthreads();                       // the previous unit's sums have been read
        s_col[wave][0][lane] = bx;
        s_col[wave][1][lane] = by;
        s_col[wave][2][lane] = bz;
        __syncthreads();
        if (threadIdx.x < kColVals) {
            const int c = threadIdx.x >> 6, l = threadIdx.x & (kWave - 1);
            a.col_part[u * kColVals + threadIdx.x] =
                ((s_col[0][c][l] + s_col[1][c][l]) + s_col[2][c][l]) + s_col[3][c][l];
        }
        if (++b == NT) {
            ++W;
            b = TPB * W;
        }
    }
    flush_sym_segment<T>(a, Wcur, wave, lane, ax, ay, az);
}

// out = (+=) pref * (row segments + column partials), fixed order.
template <int T>
__global__ __launch_bounds__(kBlock) void sym_reduce(SymArgs a, int64_t grid, double pref, double* out,
                                                     int accumulate) {
    constexpr int TPB = 4 * T, RB = kBlock * T;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n = a.in.n_trg;
    if (p >= n) return;
    const int64_t NT = a.NT, U = a.units;
    const int64_t W = p / RB, li = p % RB, b = p / kWave, l = p % kWave;
    const int64_t g0 = unit_owner(sym_off(W, NT, TPB), U, grid);
    const int64_t g1 = unit_owner(sym_off(W + 1, NT, TPB) - 1, U, grid);
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t g = g0; g <= g1; ++g) {
        const double* seg = a.row_part + (g + W) * 3 * RB;
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += seg[c * RB + li];
    }
    for (int64_t Wp = 0; Wp * TPB <= b; ++Wp) {
        const double* cp = a.col_part + (sym_off(Wp, NT, TPB) + b - TPB * Wp) * kColVals;
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += cp[c * kWave + l];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t o = c * n + p;
        out[o] = accumulate ? out[o] + pref * s[c] : pref * s[c];
    }
}

}  // namespace

int sym_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sym_main_f64<kSymT64>, kBlock, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

SymPlan plan_sym(int64_t n, int resident_blocks, int forced_grid) {
    SymPlan p{};
    p.T = kSymT64;
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
    off = align_up(off + (size_t)p.n_pad * sizeof(SrcSL64x), 256);
    p.off_aux = off;
    off = align_up(off + (size_t)p.n_pad * sizeof(int32_t), 256);
    p.off_meta = off;
    off = align_up(off + (size_t)p.NT * sizeof(SubMeta), 256);
    p.off_row = off;
    off = align_up(off + (size_t)(p.grid + p.NW) * 3 * (size_t)rb * sizeof(double), 256);
    p.off_col = off;
    off = align_up(off + (size_t)p.units * kColVals * sizeof(double), 256);
    p.total = off;
    return p;
}

hipError_t launch_sym(const SumInputs& in, const SymPlan& p, double* out, int accumulate, void* ws,
                      hipStream_t stream, const KernelTimer& timer) {
    if (in.n_trg <= 0) return hipSuccess;
    if (in.kernel != 0 || in.mixed) return hipErrorNotSupported;
    char* base = static_cast<char*>(ws);
    SymArgs a{};
    a.in = in;
    a.rec = base + p.off_rec;
    a.aux = base + p.off_aux;
    a.meta = reinterpret_cast<const SubMeta*>(base + p.off_meta);
    a.n_pad = p.n_pad;
    a.NT = p.NT;
    a.NW = p.NW;
    a.units = p.units;
    a.row_part = reinterpret_cast<double*>(base + p.off_row);
    a.col_part = reinterpret_cast<double*>(base + p.off_col);
    hipError_t e = launch_prep(in, p.n_pad, base + p.off_rec, base + p.off_aux,
                               reinterpret_cast<SubMeta*>(base + p.off_meta), stream);
    if (e != hipSuccess) return e;
    if (timer.on()) (void)hipEventRecord(timer.start, stream);
    sym_main_f64<kSymT64><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a);
    e = hipGetLastError();
    if (timer.on()) (void)hipEventRecord(timer.stop, stream);
    if (e != hipSuccess) return e;
    // the float64 sums are 4 times the bare single-layer sums (doubled positions)
    sym_reduce<kSymT64><<<dim3((unsigned)ceil_div(in.n_trg, kBlock)), dim3(kBlock), 0, stream>>>(
        a, p.grid, 0.25 * in.pref, out, accumulate);
    return hipGetLastError();
}

}  // namespace stokes
