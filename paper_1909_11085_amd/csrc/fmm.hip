// Kernel-independent fast multipole method for the single- and double-layer
// sums on a uniform octree (Sec. 3.1, "Far evaluation": the paper evaluates the
// smooth quadrature for all targets at once with a kernel-independent FMM).
//
// Plan (host, once per surface order p): the cube-surface template with p
// points per edge and the check-to-equivalent pseudo-inverses for a unit box,
// upward (check 2.95, equivalent 1.05) and downward (check 1.05, equivalent
// 2.95), from a one-sided Jacobi SVD that drops singular values below 1e-12 of
// the largest.  The kernel is homogeneous of degree -1, so at level l the
// operators are these times the box half-width h_l.  Everything is computed
// with the kernel times 8 pi mu; the prefactor is applied to the output.
//
// Evaluation (device, one stream, no host round trip):
//   leaf keys (Morton index of the leaf holding each point), radix sort,
//   gathers into leaf order (sources carry q = w f), leaf offsets by binary
//   search, per-level "has sources" / "has targets" flags;
//   upward: P2M (leaves), M2M (up to level 2): per box the check velocities
//   (LDS-staged pair sums), then per level one FP64 MFMA GEMM applies the
//   pseudo-inverse to all boxes;
//   downward, level 2 to the leaves: M2L + L2L as one GEMM per octant class
//   against precomputed translation operators (or as pair sums where the
//   interaction lists are sparse), then the pseudo-inverse GEMM;
//   L2P + P2P per chunk of up to 64 targets of a leaf, written back in the
//   caller's order.
// Every sum is taken in a fixed order (no atomics on values), so results are
// reproducible.
//
// Double-layer sources use the double-layer kernel in P2M and P2P.  Their
// field has a net flux (sum of n . q) that no single-layer density carries, so
// every box also holds a point source of that flux at its centre (velocity
// sigma r / (4 pi rho^3)); the upward equivalent density represents the
// flux-free rest, M2M sums the children's fluxes, and M2L adds the point
// source of each interaction-list box.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "fmm.hpp"
#include "p2p.hpp"
#include "spatial.hpp"

struct stokes_fmm_plan {
    int device = 0;
    int order = 0;
    int ns = 0;                 // surface points
    double* d_surf = nullptr;   // (ns, 3)
    // M2L as GEMMs: rows padded to mp, K blocks of kb (3ns densities, the
    // point-source flux, zero padding); see m2l_matrix_kernel
    int mp = 0, kb = 0;
    double* d_m2l = nullptr;    // (8 classes, kM2LBlocks, kb, mp)
    int32_t* d_il = nullptr;    // (8 classes, kILSize, 3) interaction-list offsets
    double* d_downA = nullptr;  // (mp, mp): downA[k * mp + r] = DOWN[r][k], zero padded
    double* d_upA = nullptr;    // the same for UP
};

namespace stokes {
namespace {

constexpr double kAlphaUE = 1.05, kAlphaUC = 2.95, kAlphaDE = 2.95, kAlphaDC = 1.05;
constexpr double kPinvRcond = 1e-10;
constexpr int kFBlock = 256;
constexpr int kFWaves = kFBlock / kWave;
constexpr int64_t kFMaxGrid = 1 << 16;

unsigned f_grid(int64_t units) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(units, kFMaxGrid)); }

std::vector<double> surface_points(int p) {
    std::vector<double> g(p), s;
    const double step = 2.0 / (p - 1);
    for (int i = 0; i < p; ++i) g[i] = -1.0 + i * step;
    g[p - 1] = 1.0;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k)
                if (std::min({i, j, k}) == 0 || std::max({i, j, k}) == p - 1) {
                    s.push_back(g[i]);
                    s.push_back(g[j]);
                    s.push_back(g[k]);
                }
    return s;
}

// (3 nx, 3 ny) row-major matrix of 8 pi mu times the single-layer kernel.
std::vector<double> kernel_matrix(const std::vector<double>& x, double ax, const std::vector<double>& y, double ay) {
    const int nx = (int)x.size() / 3, ny = (int)y.size() / 3;
    std::vector<double> K((size_t)9 * nx * ny, 0.0);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double r[3];
            for (int c = 0; c < 3; ++c) r[c] = ax * x[3 * i + c] - ay * y[3 * j + c];
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (!(r2 > 0.0)) continue;
            const double ri = 1.0 / sqrt(r2), ri3 = ri * ri * ri;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    K[(size_t)(3 * i + a) * 3 * ny + 3 * j + b] = (a == b ? ri : 0.0) + r[a] * r[b] * ri3;
        }
    return K;
}

// ---------------------------------------------------------------- device
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}
__device__ __forceinline__ int64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (int64_t)v;
}
__device__ __forceinline__ uint64_t morton(int64_t i, int64_t j, int64_t k) {
    return spread3((uint64_t)i) | spread3((uint64_t)j) << 1 | spread3((uint64_t)k) << 2;
}

struct FmmDev {
    int ns, n3, D;
    double c[3], R;
    const double* surf;
    const double* sx;          // sorted sources (3, n_src)
    const double* sq;
    const double* sn;          // sorted source normals (double layer), else null
    double* sig;               // per box: point-source flux (double layer), else null
    int64_t n_src;
    const double* tx;          // sorted targets (3, n_trg)
    const int32_t* tperm;      // caller's index of each sorted target
    int64_t n_trg;
    const int64_t* sofs;       // (8^D + 1) leaf offsets
    const int64_t* tofs;
    uint8_t* snz;              // per box of levels 2..D: has sources
    uint8_t* tpr;              // has targets
    double* ue;                // per box: 3 ns upward equivalent density
    double* de;                // downward
    int64_t base[kFmmMaxDepth + 2];   // first box of level l in the per-box arrays
    double pref;
    int accumulate;
    double* out;
    double* vbuf;              // check vectors times h, one column of mp per listed box
    int mp;
};

__device__ __forceinline__ void box_centre(const FmmDev& a, int l, uint64_t b, double* ctr, double& h) {
    h = a.R / (double)(1 << l);
    const int64_t idx[3] = {compact3(b), compact3(b >> 1), compact3(b >> 2)};
#pragma unroll
    for (int c = 0; c < 3; ++c) ctr[c] = (a.c[c] - a.R) + (double)(2 * idx[c] + 1) * h;
}

// 1/sqrt(r2): hardware estimate (about 24 correct bits) and one Newton step,
// ~1e-15 relative; 0 when skip.
__device__ __forceinline__ double rinv(double r2, bool skip = false) {
    const double y0 = skip ? 0.0 : __builtin_amdgcn_rsq(r2);
    return __builtin_fma(0.5 * y0, __builtin_fma(-r2, y0 * y0, 1.0), y0);
}

// 8 pi mu times the single-layer kernel applied to q: q / rho + r (r.q) / rho^3.
// MASKED: a zero-distance pair adds nothing; otherwise rho > 0 is assumed.
template <bool MASKED>
__device__ __forceinline__ void sl_pair(double rx, double ry, double rz, double qx, double qy, double qz, double* u) {
    const double r2 = __builtin_fma(rx, rx, __builtin_fma(ry, ry, rz * rz));
    const double ri = rinv(r2, MASKED && r2 == 0.0);
    const double c = __builtin_fma(rx, qx, __builtin_fma(ry, qy, rz * qz)) * (ri * ri);
    u[0] = __builtin_fma(__builtin_fma(c, rx, qx), ri, u[0]);
    u[1] = __builtin_fma(__builtin_fma(c, ry, qy), ri, u[1]);
    u[2] = __builtin_fma(__builtin_fma(c, rz, qz), ri, u[2]);
}

// 8 pi times the double-layer kernel: 6 r (r.n)(r.q) / rho^5.
template <bool MASKED>
__device__ __forceinline__ void dl_pair(double rx, double ry, double rz, double nx, double ny, double nz, double qx,
                                        double qy, double qz, double* u) {
    const double r2 = __builtin_fma(rx, rx, __builtin_fma(ry, ry, rz * rz));
    const double ri = rinv(r2, MASKED && r2 == 0.0);
    const double ri2 = ri * ri;
    const double rn = __builtin_fma(rx, nx, __builtin_fma(ry, ny, rz * nz));
    const double rq = __builtin_fma(rx, qx, __builtin_fma(ry, qy, rz * qz));
    const double c = 6.0 * rn * rq * (ri2 * ri2 * ri);
    u[0] = __builtin_fma(c, rx, u[0]);
    u[1] = __builtin_fma(c, ry, u[1]);
    u[2] = __builtin_fma(c, rz, u[2]);
}

// 8 pi times the velocity of a point source of flux sigma: 2 sigma r / rho^3.
__device__ __forceinline__ void point_source(double rx, double ry, double rz, double sigma, double* u) {
    const double r2 = __builtin_fma(rx, rx, __builtin_fma(ry, ry, rz * rz));
    if (r2 > 0.0 && sigma != 0.0) {
        const double ri = rinv(r2);
        const double c = 2.0 * sigma * (ri * ri * ri);
        u[0] = __builtin_fma(c, rx, u[0]);
        u[1] = __builtin_fma(c, ry, u[1]);
        u[2] = __builtin_fma(c, rz, u[2]);
    }
}

__global__ __launch_bounds__(kFBlock) void keys_kernel(const double* __restrict__ x, int64_t n, double c0, double c1,
                                                       double c2, double R, int D, uint64_t* __restrict__ keys,
                                                       int32_t* __restrict__ vals) {
    const double lo[3] = {c0 - R, c1 - R, c2 - R};
    const double nl = (double)(1 << D), cell = 2.0 * R / nl;
    for (int64_t i = (int64_t)blockIdx.x * kFBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kFBlock) {
        int64_t idx[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = floor((x[c * n + i] - lo[c]) / cell);
            if (!(v >= 0.0)) v = 0.0;                  // also NaN
            if (v > nl - 1.0) v = nl - 1.0;
            idx[c] = (int64_t)v;
        }
        keys[i] = morton(idx[0], idx[1], idx[2]);
        vals[i] = (int32_t)i;
    }
}

__global__ __launch_bounds__(kFBlock) void gather_kernel(const double* __restrict__ x, const double* __restrict__ f,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ nrm, int64_t n,
                                                         const int32_t* __restrict__ perm, double* __restrict__ sx,
                                                         double* __restrict__ sq, double* __restrict__ sn) {
    for (int64_t i = (int64_t)blockIdx.x * kFBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kFBlock) {
        const int64_t m = perm[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sx[c * n + i] = x[c * n + m];
            if (sq) sq[c * n + i] = w[m] * f[c * n + m];
            if (sn) sn[c * n + i] = nrm[c * n + m];
        }
    }
}

__global__ __launch_bounds__(kFBlock) void leaf_ofs_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                           int64_t n_leaves, int64_t* __restrict__ ofs) {
    for (int64_t L = (int64_t)blockIdx.x * kFBlock + threadIdx.x; L <= n_leaves; L += (int64_t)gridDim.x * kFBlock) {
        int64_t lo = 0, hi = n;                        // first key >= L
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < (uint64_t)L) lo = mid + 1; else hi = mid;
        }
        ofs[L] = lo;
    }
}

__global__ __launch_bounds__(kFBlock) void flags_leaf_kernel(FmmDev a) {
    const int64_t nl = (int64_t)1 << (3 * a.D);
    for (int64_t L = (int64_t)blockIdx.x * kFBlock + threadIdx.x; L < nl; L += (int64_t)gridDim.x * kFBlock) {
        a.snz[a.base[a.D] + L] = a.sofs[L + 1] > a.sofs[L];
        a.tpr[a.base[a.D] + L] = a.tofs[L + 1] > a.tofs[L];
    }
}

__global__ __launch_bounds__(kFBlock) void flags_up_kernel(FmmDev a, int l) {
    const int64_t nb = (int64_t)1 << (3 * l);
    for (int64_t b = (int64_t)blockIdx.x * kFBlock + threadIdx.x; b < nb; b += (int64_t)gridDim.x * kFBlock) {
        uint8_t s = 0, t = 0;
        for (int o = 0; o < 8; ++o) {
            s |= a.snz[a.base[l + 1] + 8 * b + o];
            t |= a.tpr[a.base[l + 1] + 8 * b + o];
        }
        a.snz[a.base[l] + b] = s;
        a.tpr[a.base[l] + b] = t;
    }
}

__device__ __forceinline__ void load_surface(const FmmDev& a, double* surf) {
    for (int r = threadIdx.x; r < 3 * a.ns; r += kFBlock) surf[r] = a.surf[r];
    __syncthreads();
}

// Adds the four waves' partial check vectors in a fixed order and stores h
// times the sum, zero-padded to mp rows, as the box's column of the level's
// check matrix; the pseudo-inverse is then applied to all columns at once.
__device__ __forceinline__ void store_check(const FmmDev& a, const double* part, double h, int64_t col) {
    __syncthreads();
    double* v = a.vbuf + col * a.mp;
    for (int r = threadIdx.x; r < a.mp; r += kFBlock)
        v[r] = r < a.n3 ? h * (((part[r] + part[a.n3 + r]) + part[2 * a.n3 + r]) + part[3 * a.n3 + r]) : 0.0;
    __syncthreads();
}

// Flux sum of n . q over a leaf's sources: per wave over a strided quarter,
// then the four waves in order; every thread gets the total.
__device__ __forceinline__ double leaf_flux(const FmmDev& a, int64_t m0, int64_t m1, double* red) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double f = 0.0;
    for (int64_t m = m0 + threadIdx.x; m < m1; m += kFBlock)
        f += a.sn[m] * a.sq[m] + a.sn[a.n_src + m] * a.sq[a.n_src + m] + a.sn[2 * a.n_src + m] * a.sq[2 * a.n_src + m];
    for (int o = kWave / 2; o >= 1; o >>= 1) f += __shfl_xor(f, o);
    if (lane == 0) red[wave] = f;
    __syncthreads();
    const double total = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return total;
}

constexpr int kMaxT = 8;                 // check points per lane
constexpr int kMaxNs = 6 * (kFmmMaxOrder - 1) * (kFmmMaxOrder - 1) + 2;
static_assert(kMaxNs <= kMaxT * kWave, "the surface kernels hold at most kMaxT check points per lane");

// Copies one box's surface densities (3 per point) into a wave's LDS slice.
__device__ __forceinline__ void stage_density(const FmmDev& a, const double* __restrict__ dens, double* dst,
                                              int lane) {
    for (int r = lane; r < a.n3; r += kWave) dst[r] = dens[r];
}

// Adds the single-layer velocity of a surface (points ctr + scale * template,
// the template and the staged densities q in LDS) at a lane's T check points.
template <int T>
__device__ __forceinline__ void surface_sum(const FmmDev& a, const double* surf, const double* ctr, double scale,
                                            const double* q, const double (&x)[T][3], double (&u)[T][3]) {
#pragma unroll 2
    for (int j = 0; j < a.ns; ++j) {
        const double sx = ctr[0] + scale * surf[3 * j], sy = ctr[1] + scale * surf[3 * j + 1],
                     sz = ctr[2] + scale * surf[3 * j + 2];
        const double qx = q[3 * j], qy = q[3 * j + 1], qz = q[3 * j + 2];
#pragma unroll
        for (int k = 0; k < T; ++k) sl_pair<false>(x[k][0] - sx, x[k][1] - sy, x[k][2] - sz, qx, qy, qz, u[k]);
    }
}

// Check points of a box (centre ctr, half-width h, radius scale alpha): lane
// j holds points j, j + 64, ... (T of them); lanes past the last point repeat
// it and are never stored.
template <int T>
__device__ __forceinline__ void check_points(const FmmDev& a, const double* surf, const double* ctr, double scale,
                                             int lane, double (&x)[T][3], double (&u)[T][3]) {
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int cp = min(lane + k * kWave, a.ns - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[k][c] = ctr[c] + scale * surf[3 * cp + c];
            u[k][c] = 0.0;
        }
    }
}

template <int T>
__device__ __forceinline__ void store_partial(const FmmDev& a, double* part, int wave, int lane,
                                              const double (&u)[T][3]) {
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int cp = lane + k * kWave;
        if (cp < a.ns)
#pragma unroll
            for (int c = 0; c < 3; ++c) part[wave * a.n3 + 3 * cp + c] = u[k][c];
    }
}

// Near field (P2P) and L2P, one wave per work item: up to 64 targets of one
// leaf (items are built per evaluation from the leaf offsets).  An item of
// n targets gives each target R = min(16, 64 / n) lanes; lane phase hp takes
// every R-th staged source, and the R partial sums are added in a fixed order
// at the end.  Sources are staged in LDS, up to 128 at a time: first the
// leaf's downward equivalent density (single-layer kernel), then the leaf's
// own sources (the only ones that can sit at zero distance from a target, so
// the only ones with the zero-distance mask), then the sources of the other
// 26 neighbour leaves as one run.

template <int KT> struct NearRec;
template <> struct NearRec<0> { using type = SrcSL64; };
template <> struct NearRec<1> { using type = SrcDL64; };


template <int KT>
__device__ __forceinline__ void load_source(const FmmDev& a, int64_t m, typename NearRec<KT>::type& r) {
    r.x = a.sx[m];
    r.y = a.sx[a.n_src + m];
    r.z = a.sx[2 * a.n_src + m];
    r.qx = a.sq[m];
    r.qy = a.sq[a.n_src + m];
    r.qz = a.sq[2 * a.n_src + m];
    if constexpr (KT == 1) {
        r.nx = a.sn[m];
        r.ny = a.sn[a.n_src + m];
        r.nz = a.sn[2 * a.n_src + m];
        r.pad = 0.0;
    }
}

template <typename Rec>
__device__ __forceinline__ Rec far_pad() {
    Rec r{};
    r.x = r.y = r.z = kPadPos;
    return r;
}

template <int KT, bool MASKED>
__device__ __forceinline__ void near_pair(const typename NearRec<KT>::type& s, double x, double y, double z,
                                          double* u) {
    if constexpr (KT == 0)
        sl_pair<MASKED>(x - s.x, y - s.y, z - s.z, s.qx, s.qy, s.qz, u);
    else
        dl_pair<MASKED>(x - s.x, y - s.y, z - s.z, s.nx, s.ny, s.nz, s.qx, s.qy, s.qz, u);
}

// Dynamic LDS of P2M: the template, then a workgroup tile of source records,
// which the four partial check vectors reuse once every wave is done with it.
size_t p2m_lds(int ns, int KT) {
    const size_t rec = KT ? sizeof(SrcDL64) : sizeof(SrcSL64);
    return ((size_t)((3 * ns + 1) & ~1) + std::max<size_t>(kFBlock * rec / sizeof(double), (size_t)kFWaves * 3 * ns)) *
           sizeof(double);
}
// ... of M2M: the template, then one density slice per wave (3 ns doubles),
// which the partial vectors reuse.
size_t m2m_lds(int ns) { return ((size_t)((3 * ns + 1) & ~1) + (size_t)kFWaves * 3 * ns) * sizeof(double); }

// P2M: the leaf's sources are staged 256 at a time; wave w sums its quarter
// of each tile at its T check points per lane (zero-distance mask: a point
// outside the root cube is counted in a boundary leaf and may sit anywhere).
template <int KT, int T>
__global__ __launch_bounds__(kFBlock) void p2m_kernel(FmmDev a, const int32_t* __restrict__ list,
                                                      const int64_t* __restrict__ n_listed) {
    using Rec = typename NearRec<KT>::type;
    extern __shared__ double sh[];
    double* surf = sh;
    Rec* tile = reinterpret_cast<Rec*>(surf + ((3 * a.ns + 1) & ~1));
    double* part = reinterpret_cast<double*>(tile);            // after the last tile's reads
    __shared__ double red[kFWaves];
    load_surface(a, surf);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t listed = *n_listed;
    for (int64_t i = blockIdx.x; i < listed; i += gridDim.x) {        // uniform over the workgroup
        const int64_t b = list[i];                                    // the i-th leaf holding sources
        double ctr[3], h;
        box_centre(a, a.D, b, ctr, h);
        const int64_t m0 = a.sofs[b], m1 = a.sofs[b + 1];
        const double sigma = KT == 1 ? leaf_flux(a, m0, m1, red) : 0.0;
        if (KT == 1 && threadIdx.x == 0) a.sig[a.base[a.D] + b] = sigma;
        double x[T][3], u[T][3];
        check_points<T>(a, surf, ctr, kAlphaUC * h, lane, x, u);
        for (int64_t c0 = m0; c0 < m1; c0 += kFBlock) {
            const int nb = (int)min((int64_t)kFBlock, m1 - c0);
            __syncthreads();                                        // readers of the previous tile are done
            Rec r = far_pad<Rec>();
            if ((int)threadIdx.x < nb) load_source<KT>(a, c0 + threadIdx.x, r);
            tile[threadIdx.x] = r;
            __syncthreads();
            const int j1 = min(kWave * (wave + 1), nb);
            for (int j = kWave * wave; j < j1; ++j) {
                const Rec sr = tile[j];
#pragma unroll
                for (int k = 0; k < T; ++k) near_pair<KT, true>(sr, x[k][0], x[k][1], x[k][2], u[k]);
            }
        }
        if (KT == 1 && wave == 0)
#pragma unroll
            for (int k = 0; k < T; ++k)
                point_source(x[k][0] - ctr[0], x[k][1] - ctr[1], x[k][2] - ctr[2], -sigma, u[k]);
        __syncthreads();                           // the partial vectors overwrite the tile
        store_partial<T>(a, part, wave, lane, u);
        store_check(a, part, h, i);
    }
}

// M2M: wave w takes children w and w + 4, stages each child's equivalent
// density in its own LDS slice and sums it at its T check points per lane.
template <int T>
__global__ __launch_bounds__(kFBlock) void m2m_kernel(FmmDev a, int l, const int32_t* __restrict__ list,
                                                      const int64_t* __restrict__ n_listed) {
    extern __shared__ double sh[];
    double* surf = sh;
    double* stage = surf + ((3 * a.ns + 1) & ~1);
    double* part = stage;                                      // once every wave is done with its densities
    load_surface(a, surf);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double* mine = stage + wave * a.n3;
    const int64_t listed = *n_listed;
    for (int64_t i = blockIdx.x; i < listed; i += gridDim.x) {
        const int64_t b = list[i];                                    // the i-th box holding sources
        double ctr[3], h;
        box_centre(a, l, b, ctr, h);
        double sigma = 0.0;                       // the children's fluxes, in a fixed order
        if (a.sig)
            for (int o = 0; o < 8; ++o) sigma += a.sig[a.base[l + 1] + 8 * b + o];
        if (a.sig && threadIdx.x == 0) a.sig[a.base[l] + b] = sigma;
        double x[T][3], u[T][3];
        check_points<T>(a, surf, ctr, kAlphaUC * h, lane, x, u);
        if (a.sig && wave == 0)
#pragma unroll
            for (int k = 0; k < T; ++k)
                point_source(x[k][0] - ctr[0], x[k][1] - ctr[1], x[k][2] - ctr[2], -sigma, u[k]);
        for (int o = wave; o < 8; o += kFWaves) {
            const uint64_t ch = 8 * b + o;
            if (!a.snz[a.base[l + 1] + ch]) continue;
            double cc[3], hc;
            box_centre(a, l + 1, ch, cc, hc);
            if (a.sig) {
                const double sg = a.sig[a.base[l + 1] + ch];
#pragma unroll
                for (int k = 0; k < T; ++k) point_source(x[k][0] - cc[0], x[k][1] - cc[1], x[k][2] - cc[2], sg, u[k]);
            }
            stage_density(a, a.ue + (a.base[l + 1] + ch) * a.n3, mine, lane);
            __builtin_amdgcn_wave_barrier();
            surface_sum<T>(a, surf, cc, kAlphaUE * hc, mine, x, u);
            __builtin_amdgcn_wave_barrier();   // reads of this child precede the next writes
        }
        __syncthreads();                           // the partial vectors overwrite the density slices
        store_partial<T>(a, part, wave, lane, u);
        store_check(a, part, h, i);
    }
}

// Mixed precision: float32 records of the sources' offsets from the item's
// leaf centre (all sources of the 27 leaves lie within 3 leaf widths of it).
// ---------------------------------------------------------------------------
// Near field.  L2P is a kernel of its own; the 27-leaf sums go to the
// leaf-to-leaf kernel (p2p.hip) with the lists of the uniform tree built here:
// every leaf holding targets lists its neighbours (itself included) that hold
// sources, in a fixed order.
// ---------------------------------------------------------------------------
template <bool FILL>
__global__ __launch_bounds__(kFBlock) void near_list_kernel(FmmDev a, int64_t* __restrict__ ofs,
                                                            int32_t* __restrict__ ul) {
    const int64_t nl = (int64_t)1 << (3 * a.D), nlx = (int64_t)1 << a.D;
    for (int64_t L = (int64_t)blockIdx.x * kFBlock + threadIdx.x; L < nl; L += (int64_t)gridDim.x * kFBlock) {
        int64_t n = 0;
        if (a.tofs[L + 1] > a.tofs[L]) {
            const int64_t c0 = compact3(L), c1 = compact3(L >> 1), c2 = compact3(L >> 2);
            for (int d = 0; d < 27; ++d) {
                const int64_t n0 = c0 + d / 9 - 1, n1 = c1 + (d / 3) % 3 - 1, n2 = c2 + d % 3 - 1;
                if (n0 < 0 || n1 < 0 || n2 < 0 || n0 >= nlx || n1 >= nlx || n2 >= nlx) continue;
                const uint64_t nb = morton(n0, n1, n2);
                if (a.sofs[nb + 1] == a.sofs[nb]) continue;
                if constexpr (FILL) ul[ofs[L] + n] = (int32_t)nb;
                ++n;
            }
        }
        if constexpr (!FILL) ofs[L] = n;
    }
}

// L2P: each target (leaf order) gets the single-layer field of its leaf's
// downward equivalent density, in float64 with the zero-distance mask (a
// target outside the root cube is counted in a boundary leaf and may sit
// anywhere); written (or added) in the caller's order.  The near field is
// added to it afterwards.
__global__ __launch_bounds__(kFBlock) void l2p_kernel(FmmDev a, const uint64_t* __restrict__ tkeys) {
    for (int64_t t = (int64_t)blockIdx.x * kFBlock + threadIdx.x; t < a.n_trg; t += (int64_t)gridDim.x * kFBlock) {
        const int64_t L = (int64_t)tkeys[t];
        double ctr[3], h;
        box_centre(a, a.D, L, ctr, h);
        const double sc = kAlphaDE * h;
        const double* de = a.de + (a.base[a.D] + L) * a.n3;
        const double x = a.tx[t], y = a.tx[a.n_trg + t], z = a.tx[2 * a.n_trg + t];
        double u[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < a.ns; ++k) {
            const double yx = ctr[0] + sc * a.surf[3 * k], yy = ctr[1] + sc * a.surf[3 * k + 1],
                         yz = ctr[2] + sc * a.surf[3 * k + 2];
            sl_pair<true>(x - yx, y - yy, z - yz, de[3 * k], de[3 * k + 1], de[3 * k + 2], u);
        }
        const int64_t o = a.tperm[t];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double val = a.pref * u[c];
            a.out[c * a.n_trg + o] = a.accumulate ? a.out[c * a.n_trg + o] + val : val;
        }
    }
}

// Leaves holding targets are at most min(8^D, n_trg); each lists at most 27.
int64_t max_list(int64_t n_trg, int64_t n_leaves) { return 27 * std::min(n_trg, n_leaves); }

// ---------------------------------------------------------------------------
// M2L as dense products on the FP64 matrix cores.
//
// A target box's position in its parent (octant class c = b & 7 of its
// Morton index) fixes its interaction list: 189 offsets o (source box minus
// target box, in units of the box width), the same for every box of the class
// and level.  For a unit box (half-width 1) the velocity at the downward check
// points of the target from the upward equivalent density e of the source box
// at offset o is M_o e, M_o a (3ns x 3ns) kernel matrix.  The kernel is
// homogeneous of degree -1, so at level l the check velocity is M_o e / h_l.
// Per class the plan stores A_c = [M_o1 ... M_o189 | L2L], each block with one
// more column, the velocity of a unit point source at the source box centre
// (the double layer's flux term; that entry of the gathered vector is
// sigma / h), and padded to kb columns; the last block maps the parent's
// downward equivalent density (radius 2.95 * 2h, centre offset -(2c - 1))
// to the check points.  Then per level and class the check vectors times h are
// V = A_c E, E gathered from the per-box densities, and the downward density
// is DOWN V (the h cancels).  Both products run as FP64 MFMA 16x16x4 tiles of
// 64 boxes, A and the gathered E staged through double-buffered LDS in chunks
// of 16 K rows.  Workgroup w takes class w & 7: consecutive workgroups are
// dealt round-robin to the eight XCDs, so each class's A_c stays in one XCD's
// L2.
constexpr int kILSize = 189;
constexpr int kM2LBlocks = kILSize + 1;
constexpr int kGemmNT = 64;          // boxes per tile
constexpr int kGemmKC = 16;          // K rows per LDS chunk (4 MFMA steps)
constexpr int kGemmThreads = 512;    // 8 waves: 4 column groups x 2 row halves
constexpr int kGemmBPT = kGemmKC * kGemmNT / kGemmThreads;   // B values per thread and chunk
constexpr int kM2LUnits = 4096;      // work units a level's M2L aims for (K is split to reach them)
constexpr double kM2LDenseFill = 0.35;   // below this interaction-list fill, M2L runs as pair sums
constexpr int kILCountParts = 2048;      // workgroups (partial counts) of the interaction-list count
constexpr int kM2LMinSplits = 3;     // so that a split has at most kM2LMaxSplitBlocks blocks
constexpr int kM2LMaxSplitBlocks = (kILSize + 1 + kM2LMinSplits - 1) / kM2LMinSplits;
typedef double v4d __attribute__((ext_vector_type(4)));

int pad16(int v) { return (v + 15) / 16 * 16; }

// Interaction-list offsets of class c, in the order of the enumeration:
// neighbours d of the parent (x slowest), then their children o.
void il_offsets(int c, std::vector<int32_t>& out) {
    const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz)
                for (int o = 0; o < 8; ++o) {
                    const int ox = 2 * dx + (o & 1) - cx, oy = 2 * dy + ((o >> 1) & 1) - cy,
                              oz = 2 * dz + (o >> 2) - cz;
                    if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) continue;
                    out.push_back(ox);
                    out.push_back(oy);
                    out.push_back(oz);
                }
}

// One thread per (class, block, check point, source point or the flux column):
// the 3 x 3 kernel block (or 3 x 1 point-source column) of A_c.
__global__ __launch_bounds__(kFBlock) void m2l_matrix_kernel(const double* __restrict__ surf, int ns, int mp, int kb,
                                                             const int32_t* __restrict__ il, double* __restrict__ A) {
    const int64_t per_block = (int64_t)ns * (ns + 1);
    const int64_t total = 8 * kM2LBlocks * per_block;
    for (int64_t t = (int64_t)blockIdx.x * kFBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kFBlock) {
        const int c = (int)(t / (kM2LBlocks * per_block));
        const int blk = (int)(t / per_block % kM2LBlocks);
        const int cp = (int)(t % per_block / (ns + 1)), k = (int)(t % (ns + 1));
        double ctr[3], scale;
        if (blk < kILSize) {
            for (int d = 0; d < 3; ++d) ctr[d] = 2.0 * il[(c * kILSize + blk) * 3 + d];
            scale = kAlphaUE;
        } else {
            for (int d = 0; d < 3; ++d) ctr[d] = -(2.0 * ((c >> d) & 1) - 1.0);
            scale = 2.0 * kAlphaDE;
        }
        double x[3], r[3];
        for (int d = 0; d < 3; ++d) x[d] = kAlphaDC * surf[3 * cp + d];
        double* col = A + ((int64_t)c * kM2LBlocks + blk) * kb * mp;   // column kk at col + kk * mp
        if (k < ns) {
            for (int d = 0; d < 3; ++d) r[d] = x[d] - (ctr[d] + scale * surf[3 * k + d]);
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double ri = 1.0 / sqrt(r2), ri3 = ri * ri * ri;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    col[(int64_t)(3 * k + b) * mp + 3 * cp + a] = (a == b ? ri : 0.0) + r[a] * r[b] * ri3;
        } else if (blk < kILSize) {
            for (int d = 0; d < 3; ++d) r[d] = x[d] - ctr[d];
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double ri = 1.0 / sqrt(r2);
            for (int a = 0; a < 3; ++a) col[(int64_t)(3 * ns) * mp + 3 * cp + a] = 2.0 * r[a] * (ri * ri * ri);
        }
    }
}

// Tile shape of the GEMMs for mw = 16 RB rows per workgroup: H row blocks per
// wave half, na doubles per A chunk, APT of them loaded per thread.  Up to
// order 6 a workgroup takes all mp rows; above, the rows are cut into row
// groups of mw (the register and LDS footprint of RB = 29 at most).
constexpr int kGemmMaxRB = 29;
template <int RB> struct GemmShape {
    static_assert(RB <= kGemmMaxRB, "row blocks per workgroup");
    static constexpr int mw = 16 * RB, H = (RB + 1) / 2, na = kGemmKC * mw;
    static constexpr int APT = (na + kGemmThreads - 1) / kGemmThreads;
};
// Row blocks per workgroup for mp rows, and the row groups that cover them.
int gemm_rb(int mp) {
    const int blocks = mp / 16, ng = (blocks + kGemmMaxRB - 1) / kGemmMaxRB;
    return (blocks + ng - 1) / ng;
}
__host__ __device__ inline int gemm_groups(int mp, int rb) { return (mp / 16 + rb - 1) / rb; }

// C(r0 + row, j) = A B(:, j) for the 64 columns of a tile and rows r0 ..
// r0 + mw - 1, over the K chunks chunk(0) .. chunk(n - 1) of kGemmKC rows
// each, then store(j, row, value) for the rows < nrow.  A: K x lda, k-major
// (A[k * lda + row]); rows at or past lda read as zero.
// Each chunk of A and of B goes through LDS (two buffers); chunk t + 2 is in
// flight in registers while chunk t is multiplied.  loadb(q, j, k)
// gives row k of chunk q for column j; busy(t, g) is false when chunk t is
// zero for all 16 columns of group g (that wave skips its products).  Eight
// waves: wave w owns columns 16 (w & 3) .. + 15 and the NR row blocks from
// (w >> 2) H, H = ceil(RB / 2) (NR = H for the lower half, RB - H for the
// upper: the caller picks the instance with a wave-uniform branch).  acc[i]
// holds row block (w >> 2) H + i; lane l, entry r is row (l >> 4) + 4 r and
// column 16 (w & 3) + (l & 15).
template <int RB, int NR, typename Chunk, typename LoadB, typename Busy, typename Store>
__device__ __forceinline__ void gemm_tile(const double* __restrict__ A, int lda, int r0, int64_t n, Chunk&& chunk,
                                          LoadB&& loadb, Busy&& busy, double* As, double* Bs, int nrow,
                                          Store&& store) {
    using G = GemmShape<RB>;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int cg = wave & 3, rb0 = (wave >> 2) * G::H;
    const int bj = tid >> 3, bk = tid & 7;                   // B rows bk, bk + 8, ... of column bj
    v4d acc[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
    double pa[G::APT], pb[kGemmBPT];
    auto fetch = [&](int64_t t) {
        const int64_t q = chunk(t);
        const double* Aq = A + q * kGemmKC * lda + r0;
#pragma unroll
        for (int i = 0; i < G::APT; ++i) {
            const int e = tid + i * kGemmThreads;
            const int k = e / G::mw, r = e - k * G::mw;
            pa[i] = (e < G::na && r0 + r < lda) ? Aq[k * lda + r] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kGemmBPT; ++i) pb[i] = loadb(q, bj, bk + 8 * i);
    };
    auto put = [&](int buf) {
        double* Ab = As + buf * G::na;
#pragma unroll
        for (int i = 0; i < G::APT; ++i) {
            const int e = tid + i * kGemmThreads;
            if (e < G::na) Ab[e] = pa[i];
        }
#pragma unroll
        for (int i = 0; i < kGemmBPT; ++i) Bs[buf * (kGemmKC * kGemmNT) + (bk + 8 * i) * kGemmNT + bj] = pb[i];
    };
    auto multiply = [&](int64_t t) {
        if (!busy(t, cg)) return;                                 // uniform over the wave
        const double* Ab = As + (t & 1) * G::na;
        const double* Bb = Bs + (t & 1) * (kGemmKC * kGemmNT);
#pragma unroll
        for (int st = 0; st < kGemmKC / 4; ++st) {
            const int kr = 4 * st + (lane >> 4);
            const double bv = Bb[kr * kGemmNT + 16 * cg + (lane & 15)];
            double av[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) av[i] = Ab[kr * G::mw + 16 * (rb0 + i) + (lane & 15)];
#pragma unroll
            for (int i = 0; i < NR; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv, acc[i], 0, 0, 0);
        }
    };
    // LDS holds chunks t and t + 1 (buffers t & 1 and its pair); the registers
    // hold chunk t + 2, fetched while chunk t is multiplied
    if (n > 0) {
        fetch(0);
        put(0);
    }
    if (n > 1) {
        fetch(1);
        put(1);
    }
    if (n > 2) fetch(2);
    __syncthreads();
    for (int64_t t = 0; t < n; ++t) {
        multiply(t);
        __syncthreads();                                          // every wave is done with buffer t & 1
        if (t + 2 < n) {
            // chunk t + 2 into the freed buffer: it is read after the next
            // iteration's barrier
            put((int)(t & 1));
            if (t + 3 < n) fetch(t + 3);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (rb0 + i) + (lane >> 4) + 4 * r;
            if (row < nrow) store(16 * cg + (lane & 15), row, acc[i][r]);
        }
}

// Runs gemm_tile with the row-block count of this wave's half (a scalar branch).
template <int RB, typename Chunk, typename LoadB, typename Busy, typename Store>
__device__ __forceinline__ void gemm_tile_any(const double* __restrict__ A, int lda, int r0, int64_t n, Chunk&& chunk,
                                              LoadB&& loadb, Busy&& busy, double* As, double* Bs, int nrow,
                                              Store&& store) {
    using G = GemmShape<RB>;
    if (__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave) >> 2) != 0)
        gemm_tile<RB, RB - G::H>(A, lda, r0, n, chunk, loadb, busy, As, Bs, nrow, store);
    else
        gemm_tile<RB, G::H>(A, lda, r0, n, chunk, loadb, busy, As, Bs, nrow, store);
}

struct M2LArgs {
    const double* A;           // plan's class matrices
    const int32_t* il;
    int mp;
    const int64_t* cscan;      // exclusive scan of the class-major target flags (8 * 8^(l-1)); the
                               // upward pass reuses it for the boxes holding sources
    const int64_t* ctotal;     // number of listed boxes
    const int32_t* list;       // target boxes of the level, grouped by class
    int64_t* sched;            // [0]: K splits of this level, [1]: 1 = pair sums instead of the GEMM
    int64_t* npairs;           // per workgroup of il_count_kernel: non-empty (target box,
                               // interaction-list box) pairs of the level
    double* vbuf;              // (splits, listed boxes, mp): partial check vectors times h
};

// Class-major "holds targets" flags of level l: slot (b & 7) * 8^(l-1) + (b >> 3).
__global__ __launch_bounds__(kFBlock) void class_flags_kernel(FmmDev a, int l, int64_t* __restrict__ f) {
    const int64_t nb = (int64_t)1 << (3 * l), P = nb >> 3;
    for (int64_t b = (int64_t)blockIdx.x * kFBlock + threadIdx.x; b < nb; b += (int64_t)gridDim.x * kFBlock)
        f[(b & 7) * P + (b >> 3)] = a.tpr[a.base[l] + b] ? 1 : 0;
}
__global__ __launch_bounds__(kFBlock) void class_list_kernel(FmmDev a, int l, const int64_t* __restrict__ scan,
                                                             int32_t* __restrict__ list) {
    const int64_t nb = (int64_t)1 << (3 * l), P = nb >> 3;
    for (int64_t b = (int64_t)blockIdx.x * kFBlock + threadIdx.x; b < nb; b += (int64_t)gridDim.x * kFBlock)
        if (a.tpr[a.base[l] + b]) list[scan[(b & 7) * P + (b >> 3)]] = (int32_t)b;
}

// K splits of a level: enough work units for the whole chip, at most one
// K block each.
__global__ __launch_bounds__(kWave) void m2l_sched_kernel(const int64_t* __restrict__ cscan,
                                                          const int64_t* __restrict__ ctotal, int l,
                                                          const int64_t* __restrict__ npairs, int n_parts,
                                                          int64_t* __restrict__ sched) {
    int64_t pairs = 0;                                         // the count kernel's partials
    for (int i = threadIdx.x; i < n_parts; i += kWave) pairs += npairs[i];
    for (int o = kWave / 2; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o);
    if (threadIdx.x != 0) return;
    // sparse interaction lists (few of the 189 offsets hold sources) run as
    // pair sums: the GEMM would multiply mostly zero blocks
    sched[1] = (double)pairs < kM2LDenseFill * (double)*ctotal * kILSize ? 1 : 0;
    const int64_t P = (int64_t)1 << (3 * (l - 1));
    int64_t tiles = 0;
    for (int c = 0; c < 8; ++c) {
        const int64_t n = (c < 7 ? cscan[(c + 1) * P] : *ctotal) - cscan[c * P];
        tiles += (n + kGemmNT - 1) / kGemmNT;
    }
    int64_t S = tiles > 0 ? (kM2LUnits + tiles - 1) / tiles : 1;
    sched[0] = S < kM2LMinSplits ? kM2LMinSplits : (S > kM2LBlocks ? kM2LBlocks : S);
}

// Counts the non-empty interaction-list boxes of the listed target boxes: one
// wave per box, lane k checking offsets k, k + 64, k + 128; one partial count
// per workgroup.
__global__ __launch_bounds__(kFBlock) void il_count_kernel(FmmDev a, M2LArgs g, int l) {
    __shared__ int64_t red[kFWaves];
    const int64_t n = *g.ctotal, nbx = (int64_t)1 << l;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    int64_t cnt = 0;
    for (int64_t i = ((int64_t)blockIdx.x * kFBlock + threadIdx.x) / kWave; i < n;
         i += (int64_t)gridDim.x * (kFBlock / kWave)) {                      // uniform over the wave
        const int64_t b = g.list[i];
        const int32_t* il = g.il + (b & 7) * kILSize * 3;
        const int64_t idx[3] = {compact3(b), compact3(b >> 1), compact3(b >> 2)};
        for (int k = lane; k < kILSize + kWave - 1; k += kWave) {
            bool hit = false;
            if (k < kILSize) {
                const int64_t ai[3] = {idx[0] + il[3 * k], idx[1] + il[3 * k + 1], idx[2] + il[3 * k + 2]};
                hit = ai[0] >= 0 && ai[1] >= 0 && ai[2] >= 0 && ai[0] < nbx && ai[1] < nbx && ai[2] < nbx &&
                      a.snz[a.base[l] + (int64_t)morton(ai[0], ai[1], ai[2])];
            }
            cnt += __builtin_popcountll(__ballot(hit));
        }
    }
    if (lane == 0) red[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) g.npairs[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Partial V = A_c E over K split `split` for one tile of 64 listed boxes of
// class blockIdx.x & 7 and one row group: blockIdx.x >> 3 = rg * units + u,
// u = split * tiles + tile, units = gridDim.x / (8 row groups).  K blocks whose
// source box is missing for all 64 columns are skipped.
template <int RB>
__global__ __launch_bounds__(kGemmThreads) void m2l_gemm_kernel(FmmDev a, M2LArgs g, int l) {
    using G = GemmShape<RB>;
    __shared__ double As[2 * G::na];
    __shared__ double Bs[2 * kGemmKC * kGemmNT];
    __shared__ int32_t s_act[kM2LMaxSplitBlocks + 1];          // active blocks of this split, then the count
    __shared__ int32_t s_src[kM2LMaxSplitBlocks][kGemmNT];     // their source boxes per column (-1: none)
    __shared__ uint8_t s_grp[kM2LMaxSplitBlocks][kGemmNT / 16]; // any source among 16 columns
    const int c = blockIdx.x & 7;
    const int mp = g.mp, ng = gemm_groups(mp, RB);
    const int64_t units = gridDim.x / (8 * ng), w = blockIdx.x >> 3, P = (int64_t)1 << (3 * (l - 1));
    const int rg = (int)(w / units);
    const int64_t u = w % units;
    const int64_t S = g.sched[0];
    if (rg >= ng) return;
    if (g.sched[1]) return;                                    // this level runs as pair sums
    const int64_t c0 = g.cscan[c * P], c1 = c < 7 ? g.cscan[(c + 1) * P] : *g.ctotal;
    const int64_t tiles = (c1 - c0 + kGemmNT - 1) / kGemmNT;
    // split-major: the tiles running together on one XCD share one slice of A_c in its L2
    const int64_t split = tiles > 0 ? u / tiles : S, tile = tiles > 0 ? u % tiles : 0;
    if (split >= S) return;                                    // uniform over the workgroup
    const int64_t col0 = c0 + tile * kGemmNT;
    const int blk0 = (int)(split * kM2LBlocks / S), blk1 = (int)((split + 1) * kM2LBlocks / S);
    const int64_t nbx = (int64_t)1 << l;
    const int32_t* il = g.il + c * kILSize * 3;
    // source box of block blk for column j (-1: none); the last block is the
    // parent's L2L, present from level 3 on
    auto source = [&](int blk, int j) -> int64_t {
        if (col0 + j >= c1) return -1;
        const int64_t b = g.list[col0 + j];
        if (blk == kILSize) return l > 2 ? (b >> 3) : -1;
        const int64_t ai[3] = {compact3(b) + il[3 * blk], compact3(b >> 1) + il[3 * blk + 1],
                               compact3(b >> 2) + il[3 * blk + 2]};
        if (ai[0] < 0 || ai[1] < 0 || ai[2] < 0 || ai[0] >= nbx || ai[1] >= nbx || ai[2] >= nbx) return -1;
        const int64_t box = (int64_t)morton(ai[0], ai[1], ai[2]);
        return a.snz[a.base[l] + box] ? box : -1;
    };
    {
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        for (int blk = blk0 + wave; blk < blk1; blk += kGemmThreads / kWave) {   // lane = column
            const int64_t src = source(blk, lane);
            s_src[blk - blk0][lane] = (int32_t)src;
            const uint64_t m = __ballot(src >= 0);
            if (lane == 0) {
                s_act[blk - blk0] = m != 0 ? 1 : 0;
                for (int gq = 0; gq < kGemmNT / 16; ++gq) s_grp[blk - blk0][gq] = ((m >> (16 * gq)) & 0xffffull) != 0;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {                                    // active blocks (relative to blk0), in order
        int n = 0;
        for (int k = 0; k < blk1 - blk0; ++k)
            if (s_act[k]) s_act[n++] = k;
        s_act[kM2LMaxSplitBlocks] = n;
    }
    __syncthreads();
    const int nact = s_act[kM2LMaxSplitBlocks];
    const int cpb = mp / kGemmKC;                              // chunks per K block (the plan has kb == mp)
    const double inv_h = (double)(1 << l) / a.R;
    auto chunk = [&](int64_t t) {
        const int ti = (int)t;
        return (int64_t)(blk0 + s_act[ti / cpb]) * cpb + ti % cpb;
    };
    auto busy = [&](int64_t t, int gq) { return s_grp[s_act[(int)t / cpb]][gq] != 0; };
    auto loadb = [&](int64_t q, int j, int bk) -> double {
        const int qi = (int)q, blk = qi / cpb, kk = (qi % cpb) * kGemmKC + bk;
        const int32_t src = s_src[blk - blk0][j];
        if (src < 0) return 0.0;
        if (blk == kILSize) return kk < a.n3 ? a.de[(a.base[l - 1] + src) * a.n3 + kk] : 0.0;
        const int64_t box = a.base[l] + src;
        if (kk < a.n3) return a.ue[box * a.n3 + kk];
        return (kk == a.n3 && a.sig) ? a.sig[box] * inv_h : 0.0;
    };
    const int64_t listed = *g.ctotal;
    double* part = g.vbuf + split * listed * mp;
    const int r0 = rg * G::mw;
    gemm_tile_any<RB>(g.A + (int64_t)c * kM2LBlocks * mp * mp, mp, r0, (int64_t)nact * cpb, chunk, loadb, busy, As,
                      Bs, mp - r0, [&](int j, int row, double v) {
                          if (col0 + j < c1) part[(col0 + j) * mp + r0 + row] = v;
                      });
}

// Dynamic LDS of the pair-sum M2L kernel, in doubles: the template, then one
// density slice of 3 ns doubles per wave, which the partial check vectors
// reuse once every wave is done with its sources.
size_t m2l_lds(int ns) { return ((size_t)((3 * ns + 1) & ~1) + (size_t)kFWaves * 3 * ns) * sizeof(double); }

// M2L as pair sums, for levels whose interaction lists are sparse: per target
// box, the interaction-list boxes that hold sources (plus L2L from the parent,
// levels > 2) summed at its check points; the check vector goes to the box's
// column of the level's check matrix (the same column the GEMM would fill).
// Lane j holds check points j, j + 64, ... (T of them) in registers; wave w
// takes every fourth source box, stages its equivalent sources in its own LDS
// slice and reads them back by broadcast.
template <int T>
__global__ __launch_bounds__(kFBlock) void m2l_pairs_kernel(FmmDev a, M2LArgs g, int l) {
    extern __shared__ double sh[];
    if (!g.sched[1]) return;                                   // this level runs as a GEMM
    double* surf = sh;
    double* rest = surf + ((3 * a.ns + 1) & ~1);               // 16-byte aligned
    double* part = rest;
    load_surface(a, surf);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double* mine = rest + wave * a.n3;
    const int64_t np = (int64_t)1 << (l - 1), listed = *g.ctotal;
    // the listed target boxes one after another (the list is compact, so the
    // workgroups share the boxes evenly whatever the tree's occupancy); box i
    // of the list owns column i of the check matrix
    for (int64_t i = blockIdx.x; i < listed; i += gridDim.x) {
        const int64_t b = g.list[i];
        double ctr[3], h;
        box_centre(a, l, b, ctr, h);
        const int64_t idx[3] = {compact3(b), compact3(b >> 1), compact3(b >> 2)};
        const uint64_t p = b >> 3;
        const int64_t pidx[3] = {compact3(p), compact3(p >> 1), compact3(p >> 2)};
        double x[T][3], u[T][3];
        check_points<T>(a, surf, ctr, kAlphaDC * h, lane, x, u);
        int item = 0;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    const int64_t pn[3] = {pidx[0] + dx, pidx[1] + dy, pidx[2] + dz};
                    if (pn[0] < 0 || pn[1] < 0 || pn[2] < 0 || pn[0] >= np || pn[1] >= np || pn[2] >= np) continue;
                    for (int o = 0; o < 8; ++o) {
                        const int64_t ai[3] = {2 * pn[0] + (o & 1), 2 * pn[1] + ((o >> 1) & 1), 2 * pn[2] + (o >> 2)};
                        if (llabs(ai[0] - idx[0]) <= 1 && llabs(ai[1] - idx[1]) <= 1 && llabs(ai[2] - idx[2]) <= 1)
                            continue;                      // a neighbour: near field
                        const uint64_t ab = morton(ai[0], ai[1], ai[2]);
                        if (!a.snz[a.base[l] + ab]) continue;
                        if (item++ % kFWaves != wave) continue;
                        double ac[3], ha;
                        box_centre(a, l, ab, ac, ha);
                        if (a.sig) {
                            const double sg = a.sig[a.base[l] + ab];
#pragma unroll
                            for (int k = 0; k < T; ++k)
                                point_source(x[k][0] - ac[0], x[k][1] - ac[1], x[k][2] - ac[2], sg, u[k]);
                        }
                        stage_density(a, a.ue + (a.base[l] + ab) * a.n3, mine, lane);
                        __builtin_amdgcn_wave_barrier();
                        surface_sum<T>(a, surf, ac, kAlphaUE * ha, mine, x, u);
                        __builtin_amdgcn_wave_barrier();   // reads of this box precede the next writes
                    }
                }
        if (l > 2 && item++ % kFWaves == wave) {
            double pc[3], hp;
            box_centre(a, l - 1, p, pc, hp);
            stage_density(a, a.de + (a.base[l - 1] + p) * a.n3, mine, lane);
            __builtin_amdgcn_wave_barrier();
            surface_sum<T>(a, surf, pc, kAlphaDE * hp, mine, x, u);
        }
        __syncthreads();                           // the partial vectors overwrite the staging slices
        store_partial<T>(a, part, wave, lane, u);
        store_check(a, part, h, i);
    }
}

// Adds the K-split partials of every listed box into split 0, in split order.
__global__ __launch_bounds__(kFBlock) void m2l_reduce_kernel(M2LArgs g) {
    const int64_t n = *g.ctotal * g.mp, S = g.sched[0];
    if (g.sched[1]) return;
    for (int64_t e = (int64_t)blockIdx.x * kFBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kFBlock) {
        double v = g.vbuf[e];
        for (int64_t sp = 1; sp < S; ++sp) v += g.vbuf[sp * n + e];
        g.vbuf[e] = v;
    }
}

// K splits of a level's pseudo-inverse product: a tile's K chunks run one
// after another on one workgroup, so a level with few tiles splits K until
// it has about kApplyUnits work units (at most one chunk per split).
constexpr int kApplyUnits = 512;
constexpr int kApplyReduceGrid = 1024;
__device__ __forceinline__ int64_t apply_splits(int64_t tiles, int64_t nk) {
    return tiles > 0 ? min(nk, max((int64_t)1, (int64_t)kApplyUnits / tiles)) : 1;
}

// out[list[j]] = OP V(:, j) for the listed boxes (OP padded to mp x mp,
// k-major; out rows n3 per box): the pseudo-inverse of a whole level.
// Workgroup rg * units + u (units = gridDim.x / row groups) takes row group
// rg of tile u / S, K split u % S; with one split the tile writes out, with
// more each split writes its partial (apply_reduce_kernel adds them).
template <int RB>
__global__ __launch_bounds__(kGemmThreads) void apply_gemm_kernel(FmmDev a, M2LArgs g, const double* __restrict__ op,
                                                                  double* __restrict__ out, double* __restrict__ part) {
    using G = GemmShape<RB>;
    __shared__ double As[2 * G::na];
    __shared__ double Bs[2 * kGemmKC * kGemmNT];
    const int mp = a.mp, ng = gemm_groups(mp, RB);
    const int64_t n = *g.ctotal, nk = mp / kGemmKC;
    const int64_t tiles = (n + kGemmNT - 1) / kGemmNT, S = apply_splits(tiles, nk);
    const int64_t units = gridDim.x / ng, u = blockIdx.x % units;
    const int rg = (int)(blockIdx.x / units);
    if (rg >= ng || u >= tiles * S) return;                       // uniform over the workgroup
    const int64_t col0 = (u / S) * kGemmNT, sp = u % S;
    const int64_t k0 = sp * nk / S, k1 = (sp + 1) * nk / S;
    auto chunk = [k0](int64_t t) { return k0 + t; };
    auto loadb = [&](int64_t q, int j, int bk) -> double {
        return col0 + j < n ? g.vbuf[(col0 + j) * mp + q * kGemmKC + bk] : 0.0;
    };
    auto busy = [](int64_t, int) { return true; };
    const int32_t* list = g.list;
    const int r0 = rg * G::mw;
    gemm_tile_any<RB>(op, mp, r0, k1 - k0, chunk, loadb, busy, As, Bs, a.n3 - r0, [&](int j, int row, double v) {
        if (col0 + j >= n) return;
        if (S == 1) out[(int64_t)list[col0 + j] * a.n3 + r0 + row] = v;
        else part[(sp * n + col0 + j) * a.n3 + r0 + row] = v;
    });
}

// The split partials of apply_gemm_kernel added in split order.
__global__ __launch_bounds__(kFBlock) void apply_reduce_kernel(FmmDev a, M2LArgs g, int nk,
                                                               const double* __restrict__ part,
                                                               double* __restrict__ out) {
    const int64_t n = *g.ctotal;
    const int64_t S = apply_splits((n + kGemmNT - 1) / kGemmNT, nk);
    if (S == 1) return;
    const int64_t m = n * a.n3;
    for (int64_t e = (int64_t)blockIdx.x * kFBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kFBlock) {
        double v = part[e];
        for (int64_t sp = 1; sp < S; ++sp) v += part[sp * m + e];
        out[(int64_t)g.list[e / a.n3] * a.n3 + e % a.n3] = v;
    }
}

// Boxes of level l that hold sources, in index order: flags, then (after a
// scan) the list.  The flags pass also sets the flux of the boxes without
// sources to zero (P2M and M2M visit only the listed boxes; M2M adds the flux
// of all eight children).
__global__ __launch_bounds__(kFBlock) void src_flags_kernel(FmmDev a, int l, int64_t* __restrict__ f) {
    const int64_t nb = (int64_t)1 << (3 * l);
    for (int64_t b = (int64_t)blockIdx.x * kFBlock + threadIdx.x; b < nb; b += (int64_t)gridDim.x * kFBlock) {
        const bool has = a.snz[a.base[l] + b] != 0;
        f[b] = has ? 1 : 0;
        if (!has && a.sig) a.sig[a.base[l] + b] = 0.0;
    }
}
__global__ __launch_bounds__(kFBlock) void src_list_kernel(FmmDev a, int l, const int64_t* __restrict__ scan,
                                                           int32_t* __restrict__ list) {
    const int64_t nb = (int64_t)1 << (3 * l);
    for (int64_t b = (int64_t)blockIdx.x * kFBlock + threadIdx.x; b < nb; b += (int64_t)gridDim.x * kFBlock)
        if (a.snz[a.base[l] + b]) list[scan[b]] = (int32_t)b;
}

// Calls f(std::integral_constant<int, T>) for check points per lane T
// (1 .. kMaxT), and for the GEMM row blocks per workgroup that gemm_rb gives
// at the orders of the plan.
template <typename F>
void with_T(int T, F&& f) {
    switch (T) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        default: f(std::integral_constant<int, 8>{}); break;
    }
}
static_assert(kMaxT == 8, "with_T covers 1 .. kMaxT");
template <typename F>
bool with_rb(int rb, F&& f) {
    switch (rb) {                       // orders 2 .. 10: mp / 16 = 2, 5, 11, 19, 29, 41, 56, 73, 92
        case 2: f(std::integral_constant<int, 2>{}); return true;
        case 5: f(std::integral_constant<int, 5>{}); return true;
        case 11: f(std::integral_constant<int, 11>{}); return true;
        case 19: f(std::integral_constant<int, 19>{}); return true;
        case 21: f(std::integral_constant<int, 21>{}); return true;    // 41 in 2 groups
        case 23: f(std::integral_constant<int, 23>{}); return true;    // 92 in 4
        case 25: f(std::integral_constant<int, 25>{}); return true;    // 73 in 3
        case 28: f(std::integral_constant<int, 28>{}); return true;    // 56 in 2
        case 29: f(std::integral_constant<int, 29>{}); return true;
        default: return false;
    }
}

struct FmmLayout {
    int64_t nbox = 0, n_leaves = 0;
    int64_t base[kFmmMaxDepth + 2] = {};
    SortLayout sort;
    size_t off_skeys, off_svals, off_tkeys, off_tvals, off_sort, off_sx, off_sq, off_sn, off_tx, off_sofs, off_tofs,
        off_snz, off_tpr, off_sig, off_ue, off_de, off_uofs, off_scan, off_ul, off_p2p, off_cflag, off_cscan,
        off_ctotal, off_clist, off_sched, off_vbuf, off_apart, total;
};

FmmLayout fmm_layout(int ns, int64_t n_src, int64_t n_trg, int D) {
    const int mp = pad16(3 * ns);
    FmmLayout L;
    int64_t acc = 0;
    for (int l = 2; l <= D; ++l) {
        L.base[l] = acc;
        acc += (int64_t)1 << (3 * l);
    }
    L.nbox = acc;
    L.n_leaves = (int64_t)1 << (3 * D);
    L.sort = sort_layout(std::max(n_src, n_trg));
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return at;
    };
    L.off_skeys = take((size_t)n_src * 8);
    L.off_svals = take((size_t)n_src * 4);
    L.off_tkeys = take((size_t)n_trg * 8);
    L.off_tvals = take((size_t)n_trg * 4);
    L.off_sort = take(L.sort.total);
    L.off_sx = take((size_t)3 * n_src * 8);
    L.off_sq = take((size_t)3 * n_src * 8);
    L.off_sn = take((size_t)3 * n_src * 8);
    L.off_tx = take((size_t)3 * n_trg * 8);
    L.off_sofs = take((size_t)(L.n_leaves + 1) * 8);
    L.off_tofs = take((size_t)(L.n_leaves + 1) * 8);
    L.off_snz = take((size_t)L.nbox);
    L.off_tpr = take((size_t)L.nbox);
    L.off_sig = take((size_t)L.nbox * 8);
    L.off_ue = take((size_t)L.nbox * 3 * ns * 8);
    L.off_de = take((size_t)L.nbox * 3 * ns * 8);
    // near field: the leaves' lists (offsets, entries) and the leaf-to-leaf
    // sum's workspace (sized for the largest record of either kernel and precision)
    L.off_uofs = take((size_t)(L.n_leaves + 1) * 8);
    L.off_scan = take((size_t)scan_tmp_count(L.n_leaves) * 8);
    L.off_ul = take((size_t)max_list(n_trg, L.n_leaves) * 4);
    size_t p2p = 0;
    for (int kt = 0; kt < 2; ++kt)
        for (int mx = 0; mx < 2; ++mx)
            p2p = std::max(p2p, p2p_workspace_bytes(kt, mx, n_src, n_trg, (int32_t)L.n_leaves));
    L.off_p2p = take(p2p);
    L.off_cflag = take((size_t)L.n_leaves * 8);
    L.off_cscan = take((size_t)scan_tmp_count(L.n_leaves) * 8);
    L.off_ctotal = take(8);
    L.off_clist = take((size_t)L.n_leaves * 4);
    L.off_sched = take(16 + 8 * kILCountParts);   // splits, mode, partial interaction pair counts
    // K-split partials: splits x listed boxes <= 3 listed + 64 (units + 8)
    L.off_vbuf = take((size_t)(kM2LMinSplits * std::min(L.n_leaves, std::max<int64_t>({n_src, n_trg, 1})) +
                               kGemmNT * (kM2LUnits + 8)) *
                      mp * 8);
    // split partials of the pseudo-inverse products: S x listed <= kApplyUnits x 64 columns when S > 1
    L.off_apart = take((size_t)kApplyUnits * kGemmNT * 3 * ns * 8);
    L.total = off;
    return L;
}

}  // namespace

// ---------------------------------------------------------------- host
namespace {
// Sense-reversing barrier for the Jacobi rounds (threads spin, yielding).
struct RoundBarrier {
    explicit RoundBarrier(int n) : n_(n) {}
    void wait() {
        const int g = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
            count_.store(0, std::memory_order_relaxed);
            gen_.fetch_add(1, std::memory_order_release);
        } else {
            while (gen_.load(std::memory_order_acquire) == g) std::this_thread::yield();
        }
    }
    int n_;                                    // set before any participant arrives
    std::atomic<int> count_{0}, gen_{0};
};

// f(lo, hi) over [0, n) cut into nth contiguous ranges, one thread each; a
// range whose thread cannot be started runs on the calling thread.
template <typename F>
void parallel_ranges(int64_t n, int nth, F&& f) {
    if (nth <= 1 || n < 2 * nth) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> pool;
    std::vector<int> here;
    for (int t = 1; t < nth; ++t) {
        try {
            pool.emplace_back([&, t] { f(n * t / nth, n * (t + 1) / nth); });
        } catch (...) {
            here.push_back(t);
        }
    }
    f((int64_t)0, n / nth);
    for (int t : here) f(n * t / nth, n * (t + 1) / nth);
    for (auto& th : pool) th.join();
}
}  // namespace

void pinv_jacobi(const std::vector<double>& K, int n, double rcond, std::vector<double>& P) {
    // columns of A (a[j * n + i] = K[i][j]) are rotated until orthogonal: A V = W,
    // W's columns are sigma_j u_j; pinv = sum_j v_j w_j^T / sigma_j^2.  A sweep
    // visits every column pair once in the round-robin order of a tournament:
    // m - 1 rounds (m = n rounded up to even) of m / 2 disjoint pairs, split
    // over threads.  Rotations of disjoint pairs commute, so the result does
    // not depend on the thread count.
    std::vector<double> a((size_t)n * n), v((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[(size_t)j * n + i] = K[(size_t)i * n + j];
    for (int j = 0; j < n; ++j) v[(size_t)j * n + j] = 1.0;
    const int m = n + (n & 1);
    // A pair is left alone when its columns are orthogonal to 1e-15 or one of
    // them is below 1e-12 of the largest column norm (sqrt(smax2)): such a
    // column is rounding noise, two decades under the cutoff, and rotating it
    // against the others only stirs that noise.
    double smax2 = 0.0;
    auto rotate = [&](int p, int q) -> double {    // returns the pair's |cos| of the angle before
        double* ap = &a[(size_t)p * n];
        double* aq = &a[(size_t)q * n];
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = 0; i < n; ++i) {
            al += ap[i] * ap[i];
            be += aq[i] * aq[i];
            ga += ap[i] * aq[i];
        }
        if (ga == 0.0 || al == 0.0 || be == 0.0) return 0.0;
        const double rel = fabs(ga) / sqrt(al * be);
        if (rel <= 1e-15 || std::min(al, be) <= 1e-24 * smax2) return 0.0;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < n; ++i) {
            const double x = ap[i], y = aq[i];
            ap[i] = c * x - s * y;
            aq[i] = s * x + c * y;
        }
        double* vp = &v[(size_t)p * n];
        double* vq = &v[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - s * y;
            vq[i] = s * x + c * y;
        }
        return rel;
    };
    // position k of round r holds column (k == 0 ? 0 : 1 + (k - 1 + r) % (m - 1));
    // the pairs of a round are positions (k, m - 1 - k)
    auto column = [m](int k, int r) { return k == 0 ? 0 : 1 + (k - 1 + r) % (m - 1); };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int nth = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)hw, 16, (int64_t)(m / 2) / 16}));
    std::vector<double> worst_t(nth);
    for (int sweep = 0; sweep < 40 && m >= 2; ++sweep) {
        std::fill(worst_t.begin(), worst_t.end(), 0.0);
        smax2 = 0.0;
        for (int j = 0; j < n; ++j) {
            double c = 0.0;
            for (int i = 0; i < n; ++i) c += a[(size_t)j * n + i] * a[(size_t)j * n + i];
            smax2 = std::max(smax2, c);
        }
        RoundBarrier bar(nth);
        // the threads wait for `go`, given once the participant count is
        // final (a thread that cannot be started lowers it for this sweep)
        std::atomic<int> go{0};
        const int nth_max = nth;
        auto work = [&](int tid) {
            while (go.load(std::memory_order_acquire) == 0) std::this_thread::yield();
            double worst = 0.0;
            for (int r = 0; r < m - 1; ++r) {
                for (int k = tid; k < m / 2; k += nth) {
                    const int c0 = column(k, r), c1 = column(m - 1 - k, r);
                    const int p = std::min(c0, c1), q = std::max(c0, c1);
                    if (q >= n) continue;                  // the padding column of an odd n
                    worst = std::max(worst, rotate(p, q));
                }
                if (nth > 1) bar.wait();                   // round r's columns are final
            }
            worst_t[tid] = worst;
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nth_max; ++t) {
            try {
                pool.emplace_back(work, t);
            } catch (...) {
                break;
            }
        }
        nth = (int)pool.size() + 1;
        bar.n_ = nth;
        go.store(1, std::memory_order_release);
        work(0);
        for (auto& th : pool) th.join();
        nth = nth_max;
        if (*std::max_element(worst_t.begin(), worst_t.end()) <= 1e-14) break;
    }
    // Columns near the cutoff carry rounding noise of relative size eps
    // sigma_max / sigma_j and stay slightly non-orthogonal however many sweeps
    // run.  The kept columns J (norm above rcond times the largest) are
    // therefore inverted with their Gram matrix: with D their norms and
    // C = D^-1 W_J^T W_J D^-1 (unit diagonal; the identity for orthogonal
    // columns), pinv = V_J D^-1 C^-1 D^-1 W_J^T.  C = L L^T in order of
    // decreasing norm; a column whose pivot falls below 1e-8 lies in the span
    // of the larger ones and is dropped.
    std::vector<double> nrm(n);
    double smax = 0.0;
    for (int j = 0; j < n; ++j) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += a[(size_t)j * n + i] * a[(size_t)j * n + i];
        nrm[j] = sqrt(c);
        smax = std::max(smax, nrm[j]);
    }
    std::vector<int> J;
    for (int j = 0; j < n; ++j)
        if (nrm[j] > rcond * smax) J.push_back(j);
    std::stable_sort(J.begin(), J.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    const int r = (int)J.size();
    std::vector<double> L((size_t)r * r, 0.0), Y((size_t)r * n);
    std::vector<char> keep(r, 1);
    parallel_ranges(r, nth, [&](int64_t x0, int64_t x1) {
        for (int64_t x = x0; x < x1; ++x) {
            const double* wx = &a[(size_t)J[x] * n];
            for (int y = 0; y <= x; ++y) {
                const double* wy = &a[(size_t)J[y] * n];
                double g = 0.0;
                for (int i = 0; i < n; ++i) g += wx[i] * wy[i];
                L[(size_t)x * r + y] = g / (nrm[J[x]] * nrm[J[y]]);
            }
        }
    });
    for (int j = 0; j < r; ++j) {                       // Cholesky, lower triangle in place
        double d = L[(size_t)j * r + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * r + k] * L[(size_t)j * r + k];
        if (!(d > 1e-8)) {
            keep[j] = 0;
            for (int i = j; i < r; ++i) L[(size_t)i * r + j] = 0.0;
            continue;
        }
        const double dj = sqrt(d);
        L[(size_t)j * r + j] = dj;
        for (int i = j + 1; i < r; ++i) {
            double t = L[(size_t)i * r + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * r + k] * L[(size_t)j * r + k];
            L[(size_t)i * r + j] = t / dj;
        }
    }
    // Y = C^-1 D^-1 W_J^T by forward and back substitution (dropped rows
    // zero); the columns i of Y are independent, so threads take ranges of i
    for (int x = 0; x < r; ++x)
        for (int i = 0; i < n; ++i) Y[(size_t)x * n + i] = keep[x] ? a[(size_t)J[x] * n + i] / nrm[J[x]] : 0.0;
    parallel_ranges(n, nth, [&](int64_t i0, int64_t i1) {
        for (int x = 0; x < r; ++x) {
            if (!keep[x]) continue;
            double* yx = &Y[(size_t)x * n];
            for (int k = 0; k < x; ++k) {
                const double l = L[(size_t)x * r + k];
                if (l == 0.0) continue;
                const double* yk = &Y[(size_t)k * n];
                for (int64_t i = i0; i < i1; ++i) yx[i] -= l * yk[i];
            }
            const double inv = 1.0 / L[(size_t)x * r + x];
            for (int64_t i = i0; i < i1; ++i) yx[i] *= inv;
        }
        for (int x = r - 1; x >= 0; --x) {
            if (!keep[x]) continue;
            double* yx = &Y[(size_t)x * n];
            for (int k = x + 1; k < r; ++k) {
                const double l = L[(size_t)k * r + x];
                if (l == 0.0) continue;
                const double* yk = &Y[(size_t)k * n];
                for (int64_t i = i0; i < i1; ++i) yx[i] -= l * yk[i];
            }
            const double inv = 1.0 / L[(size_t)x * r + x];
            for (int64_t i = i0; i < i1; ++i) yx[i] *= inv;
        }
    });
    // P = sum over kept x of (v_x / d_x) y_x^T; threads take ranges of rows of P
    P.assign((size_t)n * n, 0.0);
    parallel_ranges(n, nth, [&](int64_t i0, int64_t i1) {
        for (int x = 0; x < r; ++x) {
            if (!keep[x]) continue;
            const double* vj = &v[(size_t)J[x] * n];
            const double* yx = &Y[(size_t)x * n];
            const double inv = 1.0 / nrm[J[x]];
            for (int64_t i = i0; i < i1; ++i) {
                const double vi = vj[i] * inv;
                if (vi == 0.0) continue;
                double* row = &P[(size_t)i * n];
                for (int k = 0; k < n; ++k) row[k] += vi * yx[k];
            }
        }
    });
}

int fmm_plan_build(int device, int order, stokes_fmm_plan** out, std::string& err) {
    const std::vector<double> s = surface_points(order);
    const int ns = (int)s.size() / 3, n3 = 3 * ns;
    std::vector<double> up, down;
    pinv_jacobi(kernel_matrix(s, kAlphaUC, s, kAlphaUE), n3, kPinvRcond, up);
    pinv_jacobi(kernel_matrix(s, kAlphaDC, s, kAlphaDE), n3, kPinvRcond, down);
    stokes_fmm_plan* p = new (std::nothrow) stokes_fmm_plan{};
    if (!p) {
        err = "out of host memory";
        return -2;
    }
    p->device = device;
    p->order = order;
    p->ns = ns;
    const size_t sb = s.size() * 8;
    if (hipMalloc(&p->d_surf, sb) != hipSuccess ||
        hipMemcpy(p->d_surf, s.data(), sb, hipMemcpyHostToDevice) != hipSuccess) {
        fmm_plan_free(p);
        err = "device allocation or copy failed";
        return -2;
    }
    // the pseudo-inverses, padded and k-major, and the M2L class matrices (built on the device)
    const int mp = pad16(n3), kb = pad16(n3 + 1);
    p->mp = mp;
    p->kb = kb;
    if (kb != mp) {                    // 3 ns = 6 (3 (p - 1)^2 + 1) is never a multiple of 16
        fmm_plan_free(p);
        err = "internal: M2L block size";
        return -2;
    }
    std::vector<int32_t> il;
    for (int c = 0; c < 8; ++c) il_offsets(c, il);
    std::vector<double> downA((size_t)mp * mp, 0.0), upA((size_t)mp * mp, 0.0);
    for (int r = 0; r < n3; ++r)
        for (int k = 0; k < n3; ++k) {
            downA[(size_t)k * mp + r] = down[(size_t)r * n3 + k];
            upA[(size_t)k * mp + r] = up[(size_t)r * n3 + k];
        }
    const size_t ab = (size_t)8 * kM2LBlocks * kb * mp * 8;
    hipError_t e = hipMalloc(&p->d_m2l, ab);
    if (e == hipSuccess) e = hipMalloc(&p->d_il, il.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&p->d_downA, downA.size() * 8);
    if (e == hipSuccess) e = hipMalloc(&p->d_upA, upA.size() * 8);
    if (e == hipSuccess) e = hipMemcpy(p->d_upA, upA.data(), upA.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_il, il.data(), il.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_downA, downA.data(), downA.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->d_m2l, 0, ab);
    if (e == hipSuccess) {
        const int64_t work = (int64_t)8 * kM2LBlocks * ns * (ns + 1);
        hipLaunchKernelGGL(m2l_matrix_kernel, dim3(f_grid((work + kFBlock - 1) / kFBlock)), dim3(kFBlock), 0, 0,
                           p->d_surf, ns, mp, kb, p->d_il, p->d_m2l);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess || (int)il.size() != 8 * kILSize * 3) {
        fmm_plan_free(p);
        err = "M2L operators: " + std::string(e != hipSuccess ? hipGetErrorString(e) : "interaction list size");
        return -2;
    }
    *out = p;
    return 0;
}

void fmm_plan_free(stokes_fmm_plan* p) {
    if (!p) return;
    (void)hipFree(p->d_surf);
    (void)hipFree(p->d_m2l);
    (void)hipFree(p->d_il);
    (void)hipFree(p->d_downA);
    (void)hipFree(p->d_upA);
    delete p;
}

int fmm_plan_order(const stokes_fmm_plan* p) { return p->order; }
int fmm_plan_device(const stokes_fmm_plan* p) { return p->device; }

size_t fmm_workspace_bytes(int order, int64_t n_src, int64_t n_trg, int depth) {
    const int ns = 6 * (order - 1) * (order - 1) + 2;
    return fmm_layout(ns, n_src, n_trg, depth).total;
}

hipError_t launch_fmm(const stokes_fmm_plan* plan, const FmmInputs& in, double* out, void* workspace,
                      hipStream_t st) {
    const bool dl = in.normal != nullptr;
    const int D = in.depth, ns = plan->ns;
    const FmmLayout L = fmm_layout(ns, in.n_src, in.n_trg, D);
    char* ws = static_cast<char*>(workspace);
    uint64_t* skeys = reinterpret_cast<uint64_t*>(ws + L.off_skeys);
    int32_t* svals = reinterpret_cast<int32_t*>(ws + L.off_svals);
    uint64_t* tkeys = reinterpret_cast<uint64_t*>(ws + L.off_tkeys);
    int32_t* tvals = reinterpret_cast<int32_t*>(ws + L.off_tvals);
    FmmDev a{};
    a.ns = ns;
    a.n3 = 3 * ns;
    a.D = D;
    for (int c = 0; c < 3; ++c) a.c[c] = in.centre[c];
    a.R = in.half_width;
    a.surf = plan->d_surf;
    a.sx = reinterpret_cast<double*>(ws + L.off_sx);
    a.sq = reinterpret_cast<double*>(ws + L.off_sq);
    a.sn = dl ? reinterpret_cast<double*>(ws + L.off_sn) : nullptr;
    a.sig = dl ? reinterpret_cast<double*>(ws + L.off_sig) : nullptr;
    a.n_src = in.n_src;
    a.tx = reinterpret_cast<double*>(ws + L.off_tx);
    a.tperm = tvals;
    a.n_trg = in.n_trg;
    a.sofs = reinterpret_cast<int64_t*>(ws + L.off_sofs);
    a.tofs = reinterpret_cast<int64_t*>(ws + L.off_tofs);
    a.snz = reinterpret_cast<uint8_t*>(ws + L.off_snz);
    a.tpr = reinterpret_cast<uint8_t*>(ws + L.off_tpr);
    a.ue = reinterpret_cast<double*>(ws + L.off_ue);
    a.de = reinterpret_cast<double*>(ws + L.off_de);
    for (int l = 0; l <= kFmmMaxDepth + 1; ++l) a.base[l] = L.base[std::min(l, kFmmMaxDepth + 1)];
    a.pref = in.pref;
    a.accumulate = in.accumulate;
    a.out = out;
    char* sort_ws = ws + L.off_sort;
    hipError_t e = hipSuccess;
    auto chk = [&e]() {
        if (e == hipSuccess) e = hipGetLastError();
        return e == hipSuccess;
    };
    // leaf order of sources and targets
    const unsigned gs = f_grid((in.n_src + kFBlock - 1) / kFBlock), gt = f_grid((in.n_trg + kFBlock - 1) / kFBlock);
    if (in.n_src > 0) {
        hipLaunchKernelGGL(keys_kernel, dim3(gs), dim3(kFBlock), 0, st, in.src_xyz, in.n_src, a.c[0], a.c[1], a.c[2],
                           a.R, D, skeys, svals);
        if (chk()) e = radix_sort_pairs(skeys, svals, in.n_src, 3 * D, sort_ws, L.sort, st);
        if (e == hipSuccess)
            hipLaunchKernelGGL(gather_kernel, dim3(gs), dim3(kFBlock), 0, st, in.src_xyz, in.density, in.weight,
                               in.normal, in.n_src, svals, const_cast<double*>(a.sx), const_cast<double*>(a.sq),
                               const_cast<double*>(a.sn));
        chk();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(keys_kernel, dim3(gt), dim3(kFBlock), 0, st, in.trg_xyz, in.n_trg, a.c[0], a.c[1], a.c[2],
                           a.R, D, tkeys, tvals);
        if (chk()) e = radix_sort_pairs(tkeys, tvals, in.n_trg, 3 * D, sort_ws, L.sort, st);
        if (e == hipSuccess)
            hipLaunchKernelGGL(gather_kernel, dim3(gt), dim3(kFBlock), 0, st, in.trg_xyz, nullptr, nullptr, nullptr,
                               in.n_trg, tvals, const_cast<double*>(a.tx), nullptr, nullptr);
        chk();
    }
    const unsigned gl = f_grid((L.n_leaves + 1 + kFBlock - 1) / kFBlock);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(leaf_ofs_kernel, dim3(gl), dim3(kFBlock), 0, st, skeys, in.n_src, L.n_leaves,
                           const_cast<int64_t*>(a.sofs));
        if (chk())
            hipLaunchKernelGGL(leaf_ofs_kernel, dim3(gl), dim3(kFBlock), 0, st, tkeys, in.n_trg, L.n_leaves,
                               const_cast<int64_t*>(a.tofs));
        if (chk()) hipLaunchKernelGGL(flags_leaf_kernel, dim3(gl), dim3(kFBlock), 0, st, a);
        for (int l = D - 1; l >= 2 && chk(); --l)
            hipLaunchKernelGGL(flags_up_kernel, dim3(f_grid(((int64_t)1 << (3 * l)) / kFBlock + 1)), dim3(kFBlock), 0,
                               st, a, l);
    }
    const int T = (ns + kWave - 1) / kWave;
    M2LArgs g2{};
    g2.A = plan->d_m2l;
    g2.il = plan->d_il;
    g2.mp = plan->mp;
    g2.cscan = reinterpret_cast<int64_t*>(ws + L.off_cflag);
    g2.ctotal = reinterpret_cast<int64_t*>(ws + L.off_ctotal);
    g2.list = reinterpret_cast<int32_t*>(ws + L.off_clist);
    g2.vbuf = reinterpret_cast<double*>(ws + L.off_vbuf);
    g2.sched = reinterpret_cast<int64_t*>(ws + L.off_sched);
    g2.npairs = reinterpret_cast<int64_t*>(ws + L.off_sched + 16);
    a.vbuf = g2.vbuf;
    a.mp = plan->mp;
    const int rb = gemm_rb(plan->mp), ngr = gemm_groups(plan->mp, rb);
    // OP V for the listed boxes of a level, into out (rows n3 per box)
    double* apart = reinterpret_cast<double*>(ws + L.off_apart);
    auto apply = [&](int l, const double* op, double* out) {
        // units: tiles x splits <= max(tiles, kApplyUnits), tiles at most the bound below
        const int64_t tiles_ub =
            (std::min<int64_t>((int64_t)1 << (3 * l), std::max(in.n_src, in.n_trg)) + kGemmNT - 1) / kGemmNT;
        const dim3 g((unsigned)(ngr * std::max<int64_t>(tiles_ub, kApplyUnits)));
        if (!with_rb(rb, [&](auto r) {
                hipLaunchKernelGGL(apply_gemm_kernel<decltype(r)::value>, g, dim3(kGemmThreads), 0, st, a, g2, op,
                                   out, apart);
            })) {
            e = hipErrorInvalidValue;                   // no GEMM instance for this order (not reached for 2..10)
            return false;
        }
        if (!chk()) return false;
        // a strided pass: most levels have one split, and then every workgroup just exits
        hipLaunchKernelGGL(apply_reduce_kernel, dim3(kApplyReduceGrid), dim3(kFBlock), 0, st, a, g2,
                           plan->mp / kGemmKC, apart, out);
        return chk();
    };
    // the boxes of level l holding sources: g2.list (box i of the list owns column i)
    auto list_sources = [&](int l) {
        const int64_t nb = (int64_t)1 << (3 * l);
        const unsigned gb = f_grid((nb + kFBlock - 1) / kFBlock);
        int64_t* f = const_cast<int64_t*>(g2.cscan);
        hipLaunchKernelGGL(src_flags_kernel, dim3(gb), dim3(kFBlock), 0, st, a, l, f);
        if (!chk()) return false;
        e = exclusive_scan_i64(f, nb, f, reinterpret_cast<int64_t*>(ws + L.off_cscan), const_cast<int64_t*>(g2.ctotal),
                               st);
        if (e != hipSuccess) return false;
        hipLaunchKernelGGL(src_list_kernel, dim3(gb), dim3(kFBlock), 0, st, a, l, g2.cscan,
                           const_cast<int32_t*>(g2.list));
        return chk();
    };
    // upward pass: check vectors per level, then the pseudo-inverse as one GEMM
    if (chk() && list_sources(D)) {
        const dim3 g(f_grid(L.n_leaves));
        const size_t lds = p2m_lds(ns, dl ? 1 : 0);
        with_T(T, [&](auto tc) {
            constexpr int TT = decltype(tc)::value;
            if (dl) hipLaunchKernelGGL((p2m_kernel<1, TT>), g, dim3(kFBlock), lds, st, a, g2.list, g2.ctotal);
            else hipLaunchKernelGGL((p2m_kernel<0, TT>), g, dim3(kFBlock), lds, st, a, g2.list, g2.ctotal);
        });
        if (chk()) apply(D, plan->d_upA, a.ue + L.base[D] * a.n3);
    }
    for (int l = D - 1; l >= 2 && chk(); --l) {
        if (!list_sources(l)) break;
        const dim3 g(f_grid((int64_t)1 << (3 * l)));
        const size_t lds = m2m_lds(ns);
        with_T(T, [&](auto tc) {
            hipLaunchKernelGGL(m2m_kernel<decltype(tc)::value>, g, dim3(kFBlock), lds, st, a, l, g2.list, g2.ctotal);
        });
        if (chk()) apply(l, plan->d_upA, a.ue + L.base[l] * a.n3);
    }
    for (int l = 2; l <= D && chk(); ++l) {
        const int64_t nb = (int64_t)1 << (3 * l);
        const unsigned gb = f_grid((nb + kFBlock - 1) / kFBlock);
        int64_t* cflag = const_cast<int64_t*>(g2.cscan);
        hipLaunchKernelGGL(class_flags_kernel, dim3(gb), dim3(kFBlock), 0, st, a, l, cflag);
        if (!chk()) break;
        e = exclusive_scan_i64(cflag, nb, cflag, reinterpret_cast<int64_t*>(ws + L.off_cscan),
                               const_cast<int64_t*>(g2.ctotal), st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(class_list_kernel, dim3(gb), dim3(kFBlock), 0, st, a, l, g2.cscan,
                           const_cast<int32_t*>(g2.list));
        if (!chk()) break;
        const int n_parts = (int)std::min<int64_t>(kILCountParts, (std::min<int64_t>(nb, in.n_trg) + 3) / 4);
        hipLaunchKernelGGL(il_count_kernel, dim3(n_parts), dim3(kFBlock), 0, st, a, g2, l);
        if (!chk()) break;
        hipLaunchKernelGGL(m2l_sched_kernel, dim3(1), dim3(kWave), 0, st, g2.cscan, g2.ctotal, l, g2.npairs, n_parts,
                           g2.sched);
        if (!chk()) break;
        // per class at most min(8^(l-1), n_trg) boxes in `tiles` tiles; units per
        // class = splits x tiles <= max(kM2LUnits + tiles, kM2LMinSplits x tiles)
        const int64_t tiles = (std::min<int64_t>(nb >> 3, in.n_trg) + kGemmNT - 1) / kGemmNT;
        // row groups outermost: grid = 8 classes x row groups x units
        const dim3 gm((unsigned)(8 * ngr * std::max<int64_t>(kM2LUnits + tiles, kM2LMinSplits * tiles)));
        if (!with_rb(rb, [&](auto r) {
                hipLaunchKernelGGL(m2l_gemm_kernel<decltype(r)::value>, gm, dim3(kGemmThreads), 0, st, a, g2, l);
            })) {
            e = hipErrorInvalidValue;                   // no GEMM instance for this order (not reached for 2..10)
            break;
        }
        if (!chk()) break;
        hipLaunchKernelGGL(m2l_reduce_kernel, dim3(f_grid((std::min<int64_t>(nb, in.n_trg) * plan->mp + kFBlock - 1) / kFBlock)),
                           dim3(kFBlock), 0, st, g2);
        if (!chk()) break;
        {
            const dim3 g(f_grid(nb));
            const size_t lds = m2l_lds(ns);
            with_T(T, [&](auto tc) {
                hipLaunchKernelGGL(m2l_pairs_kernel<decltype(tc)::value>, g, dim3(kFBlock), lds, st, a, g2, l);
            });
        }
        if (!chk()) break;
        if (!apply(l, plan->d_downA, a.de + L.base[l] * a.n3)) break;
    }
    if (chk()) {
        // L2P, then the near field added by the leaf-to-leaf kernel over the 27-leaf lists
        hipLaunchKernelGGL(l2p_kernel, dim3(gt), dim3(kFBlock), 0, st, a, tkeys);
        if (chk() && in.n_src > 0) {
            int64_t* uofs = reinterpret_cast<int64_t*>(ws + L.off_uofs);
            int32_t* ul = reinterpret_cast<int32_t*>(ws + L.off_ul);
            hipLaunchKernelGGL(near_list_kernel<false>, dim3(gl), dim3(kFBlock), 0, st, a, uofs, ul);
            if (chk())      // uofs[n_leaves] gets the total
                e = exclusive_scan_i64(uofs, L.n_leaves, uofs, reinterpret_cast<int64_t*>(ws + L.off_scan),
                                       uofs + L.n_leaves, st);
            if (e == hipSuccess) hipLaunchKernelGGL(near_list_kernel<true>, dim3(gl), dim3(kFBlock), 0, st, a, uofs, ul);
            if (chk()) {
                SumInputs p{};
                p.kernel = dl ? 1 : 0;
                p.mixed = in.mixed;
                p.n_src = in.n_src;
                p.src_xyz = a.sx;
                p.density = a.sq;              // q = w f, already formed: unit weights
                p.weight = nullptr;
                p.normal = a.sn;
                p.n_trg = in.n_trg;
                p.trg_xyz = a.tx;
                p.excl = 0;
                // the leaf-to-leaf kernel carries the double layer's factor 6 in its prefactor
                p.pref = dl ? 6.0 * in.pref : in.pref;
                p.trg_perm = a.tperm;
                const KernelTimer none{};
                e = launch_p2p_csr(p, (int32_t)L.n_leaves, a.sofs, a.tofs, uofs, ul, -1, out, 1, ws + L.off_p2p, st,
                                   none, false);
            }
        }
    }
    chk();
    return e;
}

}  // namespace stokes
