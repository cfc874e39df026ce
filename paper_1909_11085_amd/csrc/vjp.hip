// Adjoint (vector-Jacobian product) sums of the single- and double-layer
// kernels, float64, on the pair-sum skeleton of pairsum.hpp.
//
// Notation: a forward sum u_n = pref sum_m' K(x_n - y_m) q_m with q_m = w_m f_m
// (single layer, pref = c = 1/(8 pi mu)) or u_n = d sum_m' r (r.n_m)(r.q_m)/rho^5
// (double layer, d = 6/(8 pi)); g_n = dL/du_n.  The gradients are those of the
// definitions, differentiated by hand:
//   single layer, K(r;a,b) = [(r.b)a + (r.a)b - (a.b)r]/rho^3 - 3(r.a)(r.b)r/rho^5
//     dL/dx_n = c sum_m K(r_nm; g_n, q_m)
//     dL/df_m = c w_m sum_n S(r_nm) g_n          (S symmetric and even in r)
//     dL/dy_m = -c sum_n K(r_nm; g_n, q_m) = c sum_n K(r_mn; g_n, q_m)  (K odd)
//   double layer, G(r) = grad_r[(r.n)(r.q)(r.g)/rho^5]
//                      = [(r.q)(r.g)n + (r.n)(r.g)q + (r.n)(r.q)g]/rho^5 - 5(r.n)(r.q)(r.g) r/rho^7
//     dL/dx_n   = d sum_m G(r_nm)
//     dL/dphi_m = d w_m sum_n r_nm (r_nm.n_m)(r_nm.g_n)/rho^5
//     dL/dy_m   = -d sum_n G(r_nm)              (G even)
// Source-side gradients are transposed passes: the forward's sources act as
// targets and its targets (carrying g) as sources; when only the density
// gradient is asked for, a lighter pass skips the position terms.  For a shared point set
// with one combined position gradient, a single fused pass gives
// dL/dx_p = c sum_m [K(r_pm; g_p, q_m) + K(r_pm; q_p, g_m)] and dL/df_p.
#include <algorithm>
#include <string>

#include "../../include/stokes_mi355x.h"
#include "pairsum.hpp"
#include "vjp.hpp"

namespace stokes {
namespace {

using ps::PassArgs;
using ps::rinv;
using ps::rinv_masked;

__device__ __forceinline__ double dot3(double ax, double ay, double az, double bx, double by, double bz) {
    return __builtin_fma(ax, bx, __builtin_fma(ay, by, az * bz));
}

template <bool M>
__device__ __forceinline__ double ri_of(double r2, bool skip) {
    return M ? rinv_masked(r2, skip || r2 == 0.0) : rinv(r2);
}

__device__ __forceinline__ void out3(const PassArgs& a, double* out, int64_t n, int64_t i, double s,
                                     double vx, double vy, double vz) {
    if (!out) return;
    if (a.accumulate || out == a.force_acc) {
        out[i] += s * vx;
        out[n + i] += s * vy;
        out[2 * n + i] += s * vz;
    } else {
        out[i] = s * vx;
        out[n + i] = s * vy;
        out[2 * n + i] = s * vz;
    }
}

// ---- single layer, target side: dL/dx_n --------------------------------------
// targets: trg_xyz, tv[0] = g (3, nt); sources: src_xyz, sv[0] = density, sv[1] = weight
struct SlT {
    struct alignas(16) Rec { double x, y, z, qx, qy, qz; };
    static constexpr int NACC = 3, NT = 3;
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        const int64_t n = a.n_src;
        const double w = a.sv[1][i];
        r.x = pos[0] = a.src_xyz[i];
        r.y = pos[1] = a.src_xyz[n + i];
        r.z = pos[2] = a.src_xyz[2 * n + i];
        r.qx = w * a.sv[0][i];
        r.qy = w * a.sv[0][n + i];
        r.qz = w * a.sv[0][2 * n + i];
    }
    __device__ static void pad_rec(Rec& r) {
        r.x = r.y = r.z = kPadPos;
        r.qx = r.qy = r.qz = 0.0;
    }
    __device__ static void load_t(const PassArgs& a, int64_t i, double (&v)[NT]) {
        const int64_t n = a.n_trg;
        v[0] = a.tv[0][i]; v[1] = a.tv[0][n + i]; v[2] = a.tv[0][2 * n + i];
    }
    template <bool M>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&g)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri, ri3 = ri2 * ri;
        const double rb = dot3(dx, dy, dz, s.qx, s.qy, s.qz);
        const double ra = dot3(dx, dy, dz, g[0], g[1], g[2]);
        const double ab = dot3(g[0], g[1], g[2], s.qx, s.qy, s.qz);
        const double s1 = rb * ri3, s2 = ra * ri3;
        const double s3 = -ri3 * __builtin_fma(ra * rb, 3.0 * ri2, ab);
        acc[0] = __builtin_fma(s1, g[0], __builtin_fma(s2, s.qx, __builtin_fma(s3, dx, acc[0])));
        acc[1] = __builtin_fma(s1, g[1], __builtin_fma(s2, s.qy, __builtin_fma(s3, dy, acc[1])));
        acc[2] = __builtin_fma(s1, g[2], __builtin_fma(s2, s.qz, __builtin_fma(s3, dz, acc[2])));
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        out3(a, a.out[0], a.n_trg, i, a.pref, s[0], s[1], s[2]);
    }
};

// ---- single layer, source side: dL/df_m and dL/dy_m ----------------------------
// pass targets: the forward's sources (trg_xyz = src positions, tv[0] = density,
// tv[1] = weight); pass sources: the forward's targets (src_xyz = trg positions,
// sv[0] = g).  r = y_m - x_n.
struct SlS {
    struct alignas(16) Rec { double x, y, z, gx, gy, gz; };
    static constexpr int NACC = 6, NT = 3;
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        const int64_t n = a.n_src;
        r.x = pos[0] = a.src_xyz[i];
        r.y = pos[1] = a.src_xyz[n + i];
        r.z = pos[2] = a.src_xyz[2 * n + i];
        r.gx = a.sv[0][i];
        r.gy = a.sv[0][n + i];
        r.gz = a.sv[0][2 * n + i];
    }
    __device__ static void pad_rec(Rec& r) {
        r.x = r.y = r.z = kPadPos;
        r.gx = r.gy = r.gz = 0.0;
    }
    __device__ static void load_t(const PassArgs& a, int64_t i, double (&v)[NT]) {
        const int64_t n = a.n_trg;
        const double w = a.tv[1][i];
        v[0] = w * a.tv[0][i]; v[1] = w * a.tv[0][n + i]; v[2] = w * a.tv[0][2 * n + i];
    }
    template <bool M>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&q)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri, ri3 = ri2 * ri;
        const double ra = dot3(dx, dy, dz, s.gx, s.gy, s.gz);   // r . g_n
        const double rb = dot3(dx, dy, dz, q[0], q[1], q[2]);   // r . q_m
        const double ab = dot3(s.gx, s.gy, s.gz, q[0], q[1], q[2]);
        const double sa = ra * ri3, sb = rb * ri3;
        // S(r) g = g/rho + r (r.g)/rho^3
        acc[0] = __builtin_fma(s.gx, ri, __builtin_fma(sa, dx, acc[0]));
        acc[1] = __builtin_fma(s.gy, ri, __builtin_fma(sa, dy, acc[1]));
        acc[2] = __builtin_fma(s.gz, ri, __builtin_fma(sa, dz, acc[2]));
        // K(r; g, q)
        const double s3 = -ri3 * __builtin_fma(ra * rb, 3.0 * ri2, ab);
        acc[3] = __builtin_fma(sb, s.gx, __builtin_fma(sa, q[0], __builtin_fma(s3, dx, acc[3])));
        acc[4] = __builtin_fma(sb, s.gy, __builtin_fma(sa, q[1], __builtin_fma(s3, dy, acc[4])));
        acc[5] = __builtin_fma(sb, s.gz, __builtin_fma(sa, q[2], __builtin_fma(s3, dz, acc[5])));
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        const double w = a.tv[1][i];
        out3(a, a.out[0], a.n_trg, i, a.pref * w, s[0], s[1], s[2]);
        out3(a, a.out[1], a.n_trg, i, a.pref, s[3], s[4], s[5]);
    }
};

// ---- single layer, shared point set: dL/df_p and the total dL/dx_p ------------
// targets = sources: trg_xyz, tv[0] = g, tv[1] = density, tv[2] = weight;
// records carry (y_m, q_m, g_m) from the same arrays (sv mirrors tv).
struct SlSym {
    struct alignas(16) Rec { double x, y, z, qx, qy, qz, gx, gy, gz, pad; };
    static constexpr int NACC = 8, NT = 6;   // acc: B(3), V(3), coef of g_p, coef of q_p
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        const int64_t n = a.n_src;
        const double w = a.sv[1][i];
        r.x = pos[0] = a.src_xyz[i];
        r.y = pos[1] = a.src_xyz[n + i];
        r.z = pos[2] = a.src_xyz[2 * n + i];
        r.qx = w * a.sv[0][i];
        r.qy = w * a.sv[0][n + i];
        r.qz = w * a.sv[0][2 * n + i];
        r.gx = a.sv[2][i];
        r.gy = a.sv[2][n + i];
        r.gz = a.sv[2][2 * n + i];
        r.pad = 0.0;
    }
    __device__ static void pad_rec(Rec& r) {
        r.x = r.y = r.z = kPadPos;
        r.qx = r.qy = r.qz = r.gx = r.gy = r.gz = r.pad = 0.0;
    }
    __device__ static void load_t(const PassArgs& a, int64_t i, double (&v)[NT]) {
        const int64_t n = a.n_trg;
        const double w = a.tv[2][i];
        v[0] = a.tv[0][i]; v[1] = a.tv[0][n + i]; v[2] = a.tv[0][2 * n + i];
        v[3] = w * a.tv[1][i]; v[4] = w * a.tv[1][n + i]; v[5] = w * a.tv[1][2 * n + i];
    }
    template <bool M>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&v)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri, ri3 = ri2 * ri;
        const double rqm = dot3(dx, dy, dz, s.qx, s.qy, s.qz);
        const double rgm = dot3(dx, dy, dz, s.gx, s.gy, s.gz);
        const double rgp = dot3(dx, dy, dz, v[0], v[1], v[2]);
        const double rqp = dot3(dx, dy, dz, v[3], v[4], v[5]);
        // g_p . q_m + q_p . g_m as one chain of six products
        const double ab = __builtin_fma(v[0], s.qx, __builtin_fma(v[1], s.qy, __builtin_fma(v[2], s.qz,
                          __builtin_fma(v[3], s.gx, __builtin_fma(v[4], s.gy, v[5] * s.gz)))));
        const double sgm = rgm * ri3;
        // B += S(r) g_m
        acc[0] = __builtin_fma(s.gx, ri, __builtin_fma(sgm, dx, acc[0]));
        acc[1] = __builtin_fma(s.gy, ri, __builtin_fma(sgm, dy, acc[1]));
        acc[2] = __builtin_fma(s.gz, ri, __builtin_fma(sgm, dz, acc[2]));
        // K(r; g_p, q_m) + K(r; q_p, g_m): g_p and q_p terms as scalar coefficients
        acc[6] = __builtin_fma(rqm, ri3, acc[6]);
        acc[7] += sgm;
        const double sq = rgp * ri3, sg = rqp * ri3;
        const double cr = -ri3 * __builtin_fma(__builtin_fma(rgp, rqm, rqp * rgm), 3.0 * ri2, ab);
        acc[3] = __builtin_fma(sq, s.qx, __builtin_fma(sg, s.gx, __builtin_fma(cr, dx, acc[3])));
        acc[4] = __builtin_fma(sq, s.qy, __builtin_fma(sg, s.gy, __builtin_fma(cr, dy, acc[4])));
        acc[5] = __builtin_fma(sq, s.qz, __builtin_fma(sg, s.gz, __builtin_fma(cr, dz, acc[5])));
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        const int64_t n = a.n_trg;
        const double w = a.tv[2][i];
        out3(a, a.out[0], n, i, a.pref * w, s[0], s[1], s[2]);
        const double g[3] = {a.tv[0][i], a.tv[0][n + i], a.tv[0][2 * n + i]};
        const double q[3] = {w * a.tv[1][i], w * a.tv[1][n + i], w * a.tv[1][2 * n + i]};
        out3(a, a.out[1], n, i, a.pref, __builtin_fma(s[6], g[0], __builtin_fma(s[7], q[0], s[3])),
             __builtin_fma(s[6], g[1], __builtin_fma(s[7], q[1], s[4])),
             __builtin_fma(s[6], g[2], __builtin_fma(s[7], q[2], s[5])));
    }
};

// ---- double layer, target side: dL/dx_n ---------------------------------------
// targets: trg_xyz, tv[0] = g; sources: src_xyz, sv[0] = density, sv[1] = weight, sv[2] = normal
struct DlT {
    struct alignas(16) Rec { double x, y, z, qx, qy, qz, nx, ny, nz, pad; };
    static constexpr int NACC = 4, NT = 3;   // V(3), coefficient of g_n
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        const int64_t n = a.n_src;
        const double w = a.sv[1][i];
        r.x = pos[0] = a.src_xyz[i];
        r.y = pos[1] = a.src_xyz[n + i];
        r.z = pos[2] = a.src_xyz[2 * n + i];
        r.qx = w * a.sv[0][i];
        r.qy = w * a.sv[0][n + i];
        r.qz = w * a.sv[0][2 * n + i];
        r.nx = a.sv[2][i];
        r.ny = a.sv[2][n + i];
        r.nz = a.sv[2][2 * n + i];
        r.pad = 0.0;
    }
    __device__ static void pad_rec(Rec& r) {
        r.x = r.y = r.z = kPadPos;
        r.qx = r.qy = r.qz = r.nx = r.ny = r.nz = r.pad = 0.0;
    }
    __device__ static void load_t(const PassArgs& a, int64_t i, double (&v)[NT]) {
        const int64_t n = a.n_trg;
        v[0] = a.tv[0][i]; v[1] = a.tv[0][n + i]; v[2] = a.tv[0][2 * n + i];
    }
    // SRC: also add the source-side term r (r.n)(r.g)/rho^5 of dL/dphi into v
    template <bool M, bool SRC = false>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&g)[NT],
                                bool skip, double (&acc)[NACC], double* v = nullptr) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri, ri5 = ri2 * ri2 * ri;
        const double rn = dot3(dx, dy, dz, s.nx, s.ny, s.nz);
        const double rq = dot3(dx, dy, dz, s.qx, s.qy, s.qz);
        const double rg = dot3(dx, dy, dz, g[0], g[1], g[2]);
        const double t = rg * ri5;
        const double cn = rq * t, cq = rn * t;
        const double rnrq = rn * rq;
        acc[3] = __builtin_fma(rnrq, ri5, acc[3]);
        const double cr = (rnrq * t) * (-5.0 * ri2);
        acc[0] = __builtin_fma(cn, s.nx, __builtin_fma(cq, s.qx, __builtin_fma(cr, dx, acc[0])));
        acc[1] = __builtin_fma(cn, s.ny, __builtin_fma(cq, s.qy, __builtin_fma(cr, dy, acc[1])));
        acc[2] = __builtin_fma(cn, s.nz, __builtin_fma(cq, s.qz, __builtin_fma(cr, dz, acc[2])));
        if constexpr (SRC) {
            v[0] = __builtin_fma(cq, dx, v[0]);
            v[1] = __builtin_fma(cq, dy, v[1]);
            v[2] = __builtin_fma(cq, dz, v[2]);
        }
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        const int64_t n = a.n_trg;
        out3(a, a.out[0], n, i, a.pref, __builtin_fma(s[3], a.tv[0][i], s[0]),
             __builtin_fma(s[3], a.tv[0][n + i], s[1]), __builtin_fma(s[3], a.tv[0][2 * n + i], s[2]));
    }
};

// ---- double layer, source side: dL/dphi_m and dL/dy_m ---------------------------
// pass targets: the forward's sources (trg_xyz = src positions, tv[0] = density,
// tv[1] = weight, tv[2] = normal); pass sources: the forward's targets
// (src_xyz = trg positions, sv[0] = g).  r = y_m - x_n = -r_nm.
struct DlS {
    struct alignas(16) Rec { double x, y, z, gx, gy, gz; };
    static constexpr int NACC = 8, NT = 6;   // P(3), V(3), coef of n_m, coef of q_m
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        const int64_t n = a.n_src;
        r.x = pos[0] = a.src_xyz[i];
        r.y = pos[1] = a.src_xyz[n + i];
        r.z = pos[2] = a.src_xyz[2 * n + i];
        r.gx = a.sv[0][i];
        r.gy = a.sv[0][n + i];
        r.gz = a.sv[0][2 * n + i];
    }
    __device__ static void pad_rec(Rec& r) {
        r.x = r.y = r.z = kPadPos;
        r.gx = r.gy = r.gz = 0.0;
    }
    __device__ static void load_t(const PassArgs& a, int64_t i, double (&v)[NT]) {
        const int64_t n = a.n_trg;
        const double w = a.tv[1][i];
        v[0] = a.tv[2][i]; v[1] = a.tv[2][n + i]; v[2] = a.tv[2][2 * n + i];            // n_m
        v[3] = w * a.tv[0][i]; v[4] = w * a.tv[0][n + i]; v[5] = w * a.tv[0][2 * n + i];  // q_m
    }
    template <bool M>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&v)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri, ri5 = ri2 * ri2 * ri;
        const double rn = dot3(dx, dy, dz, v[0], v[1], v[2]);
        const double rq = dot3(dx, dy, dz, v[3], v[4], v[5]);
        const double rg = dot3(dx, dy, dz, s.gx, s.gy, s.gz);
        const double t = rg * ri5;
        const double c1 = rn * t;                 // (r.n)(r.g)/rho^5
        // P += r (r.n)(r.g)/rho^5
        acc[0] = __builtin_fma(c1, dx, acc[0]);
        acc[1] = __builtin_fma(c1, dy, acc[1]);
        acc[2] = __builtin_fma(c1, dz, acc[2]);
        // G(r): n_m and q_m terms as scalar coefficients
        acc[6] = __builtin_fma(rq, t, acc[6]);
        acc[7] += c1;
        const double rnrq = rn * rq;
        const double cg = rnrq * ri5;
        const double cr = (rnrq * t) * (-5.0 * ri2);
        acc[3] = __builtin_fma(cg, s.gx, __builtin_fma(cr, dx, acc[3]));
        acc[4] = __builtin_fma(cg, s.gy, __builtin_fma(cr, dy, acc[4]));
        acc[5] = __builtin_fma(cg, s.gz, __builtin_fma(cr, dz, acc[5]));
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        const int64_t n = a.n_trg;
        const double w = a.tv[1][i];
        // r_nm = -r: dL/dphi = -d w P, dL/dy = -d (coef_n n + coef_q q + V)
        out3(a, a.out[0], n, i, -a.pref * w, s[0], s[1], s[2]);
        const double nv[3] = {a.tv[2][i], a.tv[2][n + i], a.tv[2][2 * n + i]};
        const double q[3] = {w * a.tv[0][i], w * a.tv[0][n + i], w * a.tv[0][2 * n + i]};
        out3(a, a.out[1], n, i, -a.pref, __builtin_fma(s[6], nv[0], __builtin_fma(s[7], q[0], s[3])),
             __builtin_fma(s[6], nv[1], __builtin_fma(s[7], q[1], s[4])),
             __builtin_fma(s[6], nv[2], __builtin_fma(s[7], q[2], s[5])));
    }
};

// ---- single layer, source side, density gradient only: dL/df_m ---------------
// as SlS without the position terms
struct SlSF {
    using Rec = SlS::Rec;
    static constexpr int NACC = 3, NT = 1;
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        SlS::make_rec(a, i, r, pos);
    }
    __device__ static void pad_rec(Rec& r) { SlS::pad_rec(r); }
    __device__ static void load_t(const PassArgs&, int64_t, double (&v)[NT]) { v[0] = 0.0; }
    template <bool M>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double sa = dot3(dx, dy, dz, s.gx, s.gy, s.gz) * (ri * ri * ri);
        acc[0] = __builtin_fma(s.gx, ri, __builtin_fma(sa, dx, acc[0]));
        acc[1] = __builtin_fma(s.gy, ri, __builtin_fma(sa, dy, acc[1]));
        acc[2] = __builtin_fma(s.gz, ri, __builtin_fma(sa, dz, acc[2]));
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        out3(a, a.out[0], a.n_trg, i, a.pref * a.tv[1][i], s[0], s[1], s[2]);
    }
};

// ---- double layer, source side, density gradient only: dL/dphi_m -------------
struct DlSPhi {
    using Rec = DlS::Rec;
    static constexpr int NACC = 3, NT = 3;   // NT: n_m
    __device__ static void make_rec(const PassArgs& a, int64_t i, Rec& r, double pos[3]) {
        DlS::make_rec(a, i, r, pos);
    }
    __device__ static void pad_rec(Rec& r) { DlS::pad_rec(r); }
    __device__ static void load_t(const PassArgs& a, int64_t i, double (&v)[NT]) {
        const int64_t n = a.n_trg;
        v[0] = a.tv[2][i]; v[1] = a.tv[2][n + i]; v[2] = a.tv[2][2 * n + i];
    }
    template <bool M>
    __device__ __forceinline__ static void pair(const Rec& s, double x, double y, double z, const double (&nv)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri;
        const double rn = dot3(dx, dy, dz, nv[0], nv[1], nv[2]);
        const double rg = dot3(dx, dy, dz, s.gx, s.gy, s.gz);
        const double c1 = rn * rg * (ri2 * ri2 * ri);
        acc[0] = __builtin_fma(c1, dx, acc[0]);
        acc[1] = __builtin_fma(c1, dy, acc[1]);
        acc[2] = __builtin_fma(c1, dz, acc[2]);
    }
    __device__ static void store(const PassArgs& a, int64_t i, const double (&s)[NACC]) {
        out3(a, a.out[0], a.n_trg, i, -a.pref * a.tv[1][i], s[0], s[1], s[2]);
    }
};

// ---- double layer, target side fused with the density gradient ---------------
// One sweep over the (target, source) pairs of the target-side pass also gives,
// per source, V_m = sum_n r (r.n_m)(r.g_n)/rho^5, so that dL/dphi_m = d w_m V_m
// (its coefficient is the target side's cq).  V is summed across a wave's
// targets by a butterfly and across the workgroup's waves in LDS in a fixed
// order, then stored as the unit's partial: one slot per (target block,
// source).  The near pass adds its masked pairs' V into the slots of the
// sub-tiles it takes (each slot owned by one workgroup, after the main pass),
// and a last kernel adds the target blocks in order: deterministic, no
// atomics.

// v[i][c] over the 64 lanes of the wave: lane l returns the totals of source
// i = l / 16 (two reduce-scatter steps, then a sum over 16 lanes).
__device__ __forceinline__ void wave_sum4x3(const double (&v)[4][3], int lane, double (&out)[3]) {
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0;
    double h[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double send = b5 ? v[i][c] : v[i + 2][c];
            const double keep = b5 ? v[i + 2][c] : v[i][c];
            h[i][c] = keep + __shfl_xor(send, 32);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double send = b4 ? h[0][c] : h[1][c];
        const double keep = b4 ? h[1][c] : h[0][c];
        out[c] = keep + __shfl_xor(send, 16);
    }
#pragma unroll
    for (int m = 8; m > 0; m >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] += __shfl_xor(out[c], m);
}

// Lanes past the last target hold a copy of it (the skeleton's load_tgt);
// their target-side sums are dropped, but their source-side terms would be
// added to V, so their cotangent is set to zero (every term then vanishes).
template <int T>
__device__ __forceinline__ void zero_padding_targets(const PassArgs& a, int64_t tb, int lane,
                                                     ps::Tgt<DlT, T>& t) {
#pragma unroll
    for (int k = 0; k < T; ++k)
        if (tb + (int64_t)k * kWave + lane >= a.n_trg) t.v[k][0] = t.v[k][1] = t.v[k][2] = 0.0;
}

template <int T, int W>
__global__ __launch_bounds__(kBlock, W) void dl_fused_main(PassArgs a, double* __restrict__ vpart) {
    using P = DlT;
    using Rec = P::Rec;
    constexpr int BT = kBlock * T;
    __shared__ Rec s_rec[kTile];
    __shared__ double s_part[4][3 * kTile];      // per wave: V of each source of the chunk
    const int64_t U = a.units, C = a.chunks, G = gridDim.x;
    const int64_t u0 = ps::unit_begin(blockIdx.x, U, G), u1 = ps::unit_begin(blockIdx.x + 1, U, G);
    if (u0 >= u1) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const bool excl = a.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    ps::Tgt<P, T> t;
    bool active = false;
    int64_t tbk = -1;
    double acc[T][P::NACC];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int c = 0; c < P::NACC; ++c) acc[k][c] = 0.0;

    int64_t ub = u0 / C, c = u0 % C;
    double* sp = s_part[wave];
    for (int64_t u = u0; u < u1; ++u) {
        __syncthreads();                           // previous readers of s_rec and s_part are done
        if (ub != tbk) {
            if (tbk >= 0) ps::flush<P, T>(a, tbk, wave, lane, acc);
            tbk = ub;
            const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
            active = tb < a.n_trg;
            ps::load_tgt<P, T>(a, active ? tb : 0, lane, t);
            zero_padding_targets<T>(a, active ? tb : 0, lane, t);
#pragma unroll
            for (int k = 0; k < T; ++k)
#pragma unroll
                for (int q = 0; q < P::NACC; ++q) acc[k][q] = 0.0;
        }
        s_rec[threadIdx.x] = rec[c * kTile + threadIdx.x];
        __syncthreads();
        int64_t cn = c + 1, ubn = ub;
        if (cn == C) { cn = 0; ++ubn; }
        uint32_t flags = 0;
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            const SubMeta m = a.meta[c * 4 + s];
            bool run = active && m.count != 0;
            if (run && ps::needs_near<P, T>(t, m, excl)) {
                flags |= 1u << s;                  // its pairs (and V terms) go to the near pass
                run = false;
            }
            if (!run) {
#pragma unroll
                for (int q = 0; q < 3; ++q) sp[3 * (s * kSub + lane) + q] = 0.0;
                continue;
            }
            const Rec* base = s_rec + s * kSub;
#pragma unroll 1
            for (int j0 = 0; j0 < kSub; j0 += 4) {
                double v[4][3];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i][0] = v[i][1] = v[i][2] = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const Rec sr = base[j0 + i];
#pragma unroll
                    for (int k = 0; k < T; ++k)
                        P::template pair<false, true>(sr, t.x[k], t.y[k], t.z[k], t.v[k], false, acc[k], v[i]);
                }
                double tot[3];
                wave_sum4x3(v, lane, tot);
                // the 16 lanes of a row hold the same totals: all store (no branch)
#pragma unroll
                for (int q = 0; q < 3; ++q) sp[3 * (s * kSub + j0 + (lane >> 4)) + q] = tot[q];
            }
        }
        if (active && lane == 0) a.flags[(tbk * 4 + wave) * C + c] = (uint8_t)flags;
        __syncthreads();
        // this unit's V of source c * 256 + tid: the four waves in order, stored
        // in the slot of (target block, source); padding sources get zeros
        {
            const int64_t npad = C * kTile;
            double* vp = vpart + tbk * 3 * npad + c * kTile + threadIdx.x;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int i = 3 * threadIdx.x + q;
                vp[q * npad] = ((s_part[0][i] + s_part[1][i]) + s_part[2][i]) + s_part[3][i];
            }
        }
        c = cn;
        ub = ubn;
    }
    ps::flush<P, T>(a, tbk, wave, lane, acc);
}

// The flagged sub-tiles of dl_fused_main, with the same-group and
// zero-distance masks.  A workgroup takes the sub-tiles that any wave of its
// target block flagged (every kNearSlices-th of them, for its grid row): the
// block stages the sub-tile, each wave that flagged it runs the masked pairs
// (the others add zeros), and the four waves' V are added in a fixed order
// into the sub-tile's slots of the block's partial, which no other workgroup
// touches.
template <int T>
__global__ __launch_bounds__(kBlock) void dl_fused_near(PassArgs a, double* __restrict__ vpart) {
    using P = DlT;
    using Rec = P::Rec;
    constexpr int BT = kBlock * T;
    __shared__ Rec s_src[kSub];
    __shared__ int32_t s_grp[kSub];
    __shared__ double s_v[4][3 * kSub];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t tbk = blockIdx.x, C = a.chunks, npad = C * kTile;
    const int slice = (int)blockIdx.y;
    const int64_t tb = tbk * BT + (int64_t)wave * (kWave * T);
    const bool active = tb < a.n_trg;
    // waves of the block that hold targets (the main pass writes flag rows for those only)
    const int nw = (int)std::min<int64_t>(4, (a.n_trg - tbk * BT + kWave * T - 1) / (kWave * T));
    const bool excl = a.excl != 0;
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec);
    ps::Tgt<P, T> t;
    ps::load_tgt<P, T>(a, active ? tb : tbk * BT, lane, t);
    zero_padding_targets<T>(a, active ? tb : tbk * BT, lane, t);
    double acc[T][P::NACC];
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int q = 0; q < P::NACC; ++q) acc[k][q] = 0.0;
    const uint8_t* fl = a.flags + tbk * 4 * C;
    int n = 0;                                     // flagged sub-tiles seen (block-uniform)
    for (int64_t c0 = 0; c0 < C; c0 += kWave) {
        uint32_t any = 0, mine = 0;
        if (c0 + lane < C)
            for (int w = 0; w < nw; ++w) {
                const uint32_t f = fl[w * C + c0 + lane];
                any |= f;
                if (w == wave) mine = f;
            }
        uint64_t nz = __ballot(any != 0);          // the same in every wave
        while (nz) {
            const int l = __builtin_ctzll(nz);
            nz &= nz - 1;
            uint32_t fa = (uint32_t)__builtin_amdgcn_readlane((int)any, l);
            const uint32_t fm = (uint32_t)__builtin_amdgcn_readlane((int)mine, l);
            while (fa) {
                const int sidx = __builtin_ctz(fa);
                fa &= fa - 1;
                if (n++ % ps::kNearSlices != slice) continue;
                const int64_t sub = (c0 + l) * 4 + sidx;
                __syncthreads();                   // the previous sub-tile's readers are done
                if (threadIdx.x < kSub) {
                    s_src[threadIdx.x] = rec[sub * kSub + threadIdx.x];
                    s_grp[threadIdx.x] = a.grp[sub * kSub + threadIdx.x];
                }
                __syncthreads();
                double* sv = s_v[wave];
                if (active && ((fm >> sidx) & 1u)) {
#pragma unroll 1
                    for (int j0 = 0; j0 < kSub; j0 += 4) {
                        double v[4][3];
#pragma unroll
                        for (int i = 0; i < 4; ++i) v[i][0] = v[i][1] = v[i][2] = 0.0;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const Rec sr = s_src[j0 + i];
                            const int32_t gs = s_grp[j0 + i];
#pragma unroll
                            for (int k = 0; k < T; ++k)
                                P::template pair<true, true>(sr, t.x[k], t.y[k], t.z[k], t.v[k],
                                                             excl && gs == t.g[k], acc[k], v[i]);
                        }
                        double tot[3];
                        wave_sum4x3(v, lane, tot);
                        // the 16 lanes of a row hold the same totals: all store
#pragma unroll
                        for (int q = 0; q < 3; ++q) sv[3 * (j0 + (lane >> 4)) + q] = tot[q];
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 3; ++q) sv[3 * lane + q] = 0.0;
                }
                __syncthreads();
                if (threadIdx.x < kSub) {
                    double* vp = vpart + tbk * 3 * npad + sub * kSub + threadIdx.x;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const int i = 3 * threadIdx.x + q;
                        vp[q * npad] += ((s_v[0][i] + s_v[1][i]) + s_v[2][i]) + s_v[3][i];
                    }
                }
            }
        }
    }
    if (!active) return;                           // no barriers below
    const int64_t np = (int64_t)gridDim.x * BT;
    double* part = a.near_part + (int64_t)slice * P::NACC * np;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        const int64_t gi = tbk * BT + wave * (kWave * T) + k * kWave + lane;
#pragma unroll
        for (int q = 0; q < P::NACC; ++q) part[q * np + gi] = acc[k][q];
    }
}

// dL/dphi_m = d w_m V_m, V_m the target blocks' partials added in order
__global__ __launch_bounds__(kBlock) void dl_phi_reduce(const double* __restrict__ vpart, int64_t blocks,
                                                        int64_t npad, const double* __restrict__ weight,
                                                        double pref, double* __restrict__ out, int64_t n,
                                                        int accumulate) {
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= n) return;
    const double s = pref * weight[m];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double v = 0.0;
        for (int64_t b = 0; b < blocks; ++b) v += vpart[(b * 3 + q) * npad + m];
        const double val = s * v;
        out[q * n + m] = accumulate ? out[q * n + m] + val : val;
    }
}

// launch shapes (targets per lane, minimum waves per SIMD)
constexpr int kTSlT = 4, kWSlT = 3;
constexpr int kTSlS = 2, kWSlS = 4;
#ifndef STOKES_SYM_T
#define STOKES_SYM_T 3
#endif
#ifndef STOKES_SYM_W
#define STOKES_SYM_W 2
#endif
constexpr int kTSym = STOKES_SYM_T, kWSym = STOKES_SYM_W;
constexpr int kTDlT = 4, kWDlT = 3;
constexpr int kTDlS = 2, kWDlS = 3;
constexpr int kTSlSF = 4, kWSlSF = 4;
constexpr int kTDlSPhi = 4, kWDlSPhi = 3;
constexpr int kTDlF = 4, kWDlF = 2;

// workspace of the fused double-layer pass: the target-side pass, then the
// partials of V, (target block, 3, padded source)
size_t dl_fused_bytes(int64_t n_src, int64_t n_trg, int resident, size_t* off_v) {
    const auto p = ps::plan_pass<DlT, kTDlF>(n_src, n_trg, resident);
    const size_t off = align_up(p.total, 256);
    if (off_v) *off_v = off;
    return align_up(off + (size_t)p.blocks_x * 3 * p.n_src_pad * sizeof(double), 256);
}

}  // namespace

void vjp_resident(int n_cu, int out[kVjpPasses]) {
    out[0] = ps::resident_blocks<SlT, kTSlT, kWSlT>(n_cu);
    out[1] = ps::resident_blocks<SlS, kTSlS, kWSlS>(n_cu);
    out[2] = ps::resident_blocks<SlSym, kTSym, kWSym>(n_cu);
    out[3] = ps::resident_blocks<DlT, kTDlT, kWDlT>(n_cu);
    out[4] = ps::resident_blocks<DlS, kTDlS, kWDlS>(n_cu);
    out[5] = ps::resident_blocks<SlSF, kTSlSF, kWSlSF>(n_cu);
    out[6] = ps::resident_blocks<DlSPhi, kTDlSPhi, kWDlSPhi>(n_cu);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dl_fused_main<kTDlF, kWDlF>, kBlock, 0) !=
            hipSuccess || nb < 1)
        nb = 1;
    out[7] = nb * n_cu;
}

size_t vjp_workspace_bytes(int kernel, int64_t n_src, int64_t n_trg, const int resident[kVjpPasses]) {
    if (n_src <= 0 || n_trg <= 0) return 0;
    if (kernel == 0) {
        size_t b = ps::plan_pass<SlT, kTSlT>(n_src, n_trg, resident[0]).total;
        b = std::max(b, ps::plan_pass<SlS, kTSlS>(n_trg, n_src, resident[1]).total);
        b = std::max(b, ps::plan_pass<SlSF, kTSlSF>(n_trg, n_src, resident[5]).total);
        if (n_src == n_trg) b = std::max(b, ps::plan_pass<SlSym, kTSym>(n_src, n_trg, resident[2]).total);
        return b;
    }
    size_t b = ps::plan_pass<DlT, kTDlT>(n_src, n_trg, resident[3]).total;
    b = std::max(b, dl_fused_bytes(n_src, n_trg, resident[7], nullptr));
    b = std::max(b, ps::plan_pass<DlSPhi, kTDlSPhi>(n_trg, n_src, resident[6]).total);
    return std::max(b, ps::plan_pass<DlS, kTDlS>(n_trg, n_src, resident[4]).total);
}

static PassArgs base_args(const VjpInputs& in) {
    PassArgs a{};
    a.excl = in.excl;
    a.accumulate = in.accumulate;
    return a;
}

hipError_t launch_sl_vjp(const VjpInputs& in, const int resident[kVjpPasses], bool fused, void* ws,
                         hipStream_t stream) {
    hipError_t e = hipSuccess;
    const KernelTimer none{};
    if (fused) {
        PassArgs a = base_args(in);
        a.n_trg = a.n_src = in.n_trg;
        a.trg_xyz = a.src_xyz = in.trg_xyz;
        a.trg_group = a.src_group = in.trg_group;
        a.tv[0] = a.sv[2] = in.grad_vel;
        a.tv[1] = a.sv[0] = in.density;
        a.tv[2] = a.sv[1] = in.weight;
        a.out[0] = in.grad_density;
        a.out[1] = in.grad_trg;           // == grad_src: the total position gradient
        a.pref = in.pref;
        const auto p = ps::plan_pass<SlSym, kTSym>(in.n_src, in.n_trg, resident[2]);
        return ps::run_pass<SlSym, kTSym, kWSym>(a, p, ws, stream, none);
    }
    if (in.grad_trg) {
        PassArgs a = base_args(in);
        a.n_trg = in.n_trg;
        a.trg_xyz = in.trg_xyz;
        a.trg_group = in.trg_group;
        a.tv[0] = in.grad_vel;
        a.n_src = in.n_src;
        a.src_xyz = in.src_xyz;
        a.src_group = in.src_group;
        a.sv[0] = in.density;
        a.sv[1] = in.weight;
        a.out[0] = in.grad_trg;
        a.pref = in.pref;
        const auto p = ps::plan_pass<SlT, kTSlT>(in.n_src, in.n_trg, resident[0]);
        e = ps::run_pass<SlT, kTSlT, kWSlT>(a, p, ws, stream, none);
        if (e != hipSuccess) return e;
    }
    if (in.grad_density || in.grad_src) {
        PassArgs a = base_args(in);
        a.n_trg = in.n_src;
        a.trg_xyz = in.src_xyz;
        a.trg_group = in.src_group;
        a.tv[0] = in.density;
        a.tv[1] = in.weight;
        a.n_src = in.n_trg;
        a.src_xyz = in.trg_xyz;
        a.src_group = in.trg_group;
        a.sv[0] = in.grad_vel;
        a.out[0] = in.grad_density;
        a.out[1] = in.grad_src;
        a.pref = in.pref;
        if (in.grad_src) {
            const auto p = ps::plan_pass<SlS, kTSlS>(in.n_trg, in.n_src, resident[1]);
            e = ps::run_pass<SlS, kTSlS, kWSlS>(a, p, ws, stream, none);
        } else {
            const auto p = ps::plan_pass<SlSF, kTSlSF>(in.n_trg, in.n_src, resident[5]);
            e = ps::run_pass<SlSF, kTSlSF, kWSlSF>(a, p, ws, stream, none);
        }
    }
    return e;
}

// dL/dx (targets) and dL/dphi in one sweep over the pairs; see dl_fused_main.
static hipError_t launch_dl_fused(const VjpInputs& in, int resident, void* ws, hipStream_t stream) {
    PassArgs a = base_args(in);
    a.n_trg = in.n_trg;
    a.trg_xyz = in.trg_xyz;
    a.trg_group = in.trg_group;
    a.tv[0] = in.grad_vel;
    a.n_src = in.n_src;
    a.src_xyz = in.src_xyz;
    a.src_group = in.src_group;
    a.sv[0] = in.density;
    a.sv[1] = in.weight;
    a.sv[2] = in.normal;
    a.out[0] = in.grad_trg;
    a.pref = in.pref;
    const auto p = ps::plan_pass<DlT, kTDlF>(in.n_src, in.n_trg, resident);
    size_t off_v = 0;
    (void)dl_fused_bytes(in.n_src, in.n_trg, resident, &off_v);
    char* base = static_cast<char*>(ws);
    a.rec = base + p.off_rec;
    a.grp = reinterpret_cast<int32_t*>(base + p.off_grp);
    a.meta = reinterpret_cast<SubMeta*>(base + p.off_meta);
    a.part = reinterpret_cast<double*>(base + p.off_part);
    a.near_part = reinterpret_cast<double*>(base + p.off_near);
    a.flags = reinterpret_cast<uint8_t*>(base + p.off_flags);
    a.chunks = p.chunks;
    a.units = p.units;
    double* vpart = reinterpret_cast<double*>(base + off_v);
    ps::prep<DlT><<<dim3((unsigned)(p.n_src_pad / kBlock)), dim3(kBlock), 0, stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the main pass writes every (target block, source) slot of vpart
    dl_fused_main<kTDlF, kWDlF><<<dim3((unsigned)p.grid), dim3(kBlock), 0, stream>>>(a, vpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    dl_fused_near<kTDlF><<<dim3((unsigned)p.blocks_x, ps::kNearSlices), dim3(kBlock), 0, stream>>>(a, vpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ps::reduce<DlT, kTDlF><<<dim3((unsigned)ceil_div(a.n_trg, kBlock)), dim3(kBlock), 0, stream>>>(
        a, p.grid, p.blocks_x * (int64_t)kBlock * kTDlF);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    dl_phi_reduce<<<dim3((unsigned)ceil_div(in.n_src, kBlock)), dim3(kBlock), 0, stream>>>(
        vpart, p.blocks_x, p.n_src_pad, in.weight, in.pref, in.grad_density, in.n_src, in.accumulate);
    return hipGetLastError();
}

hipError_t launch_dl_vjp(const VjpInputs& in, const int resident[kVjpPasses], bool combined,
                         void* ws, hipStream_t stream) {
    hipError_t e = hipSuccess;
    const KernelTimer none{};
    if (in.grad_trg && in.grad_density && !in.grad_src) return launch_dl_fused(in, resident[7], ws, stream);
    if (in.grad_trg) {
        PassArgs a = base_args(in);
        a.n_trg = in.n_trg;
        a.trg_xyz = in.trg_xyz;
        a.trg_group = in.trg_group;
        a.tv[0] = in.grad_vel;
        a.n_src = in.n_src;
        a.src_xyz = in.src_xyz;
        a.src_group = in.src_group;
        a.sv[0] = in.density;
        a.sv[1] = in.weight;
        a.sv[2] = in.normal;
        a.out[0] = in.grad_trg;
        a.pref = in.pref;
        const auto p = ps::plan_pass<DlT, kTDlT>(in.n_src, in.n_trg, resident[3]);
        e = ps::run_pass<DlT, kTDlT, kWDlT>(a, p, ws, stream, none);
        if (e != hipSuccess) return e;
    }
    if (in.grad_density || in.grad_src) {
        PassArgs a = base_args(in);
        a.n_trg = in.n_src;
        a.trg_xyz = in.src_xyz;
        a.trg_group = in.src_group;
        a.tv[0] = in.density;
        a.tv[1] = in.weight;
        a.tv[2] = in.normal;
        a.n_src = in.n_trg;
        a.src_xyz = in.trg_xyz;
        a.src_group = in.trg_group;
        a.sv[0] = in.grad_vel;
        a.out[0] = in.grad_density;
        a.out[1] = in.grad_src;
        a.pref = in.pref;
        // one array for both position gradients: the target side is already
        // in it, so the source side adds to it
        if (combined) a.force_acc = in.grad_src;
        if (in.grad_src) {
            const auto p = ps::plan_pass<DlS, kTDlS>(in.n_trg, in.n_src, resident[4]);
            e = ps::run_pass<DlS, kTDlS, kWDlS>(a, p, ws, stream, none);
        } else {
            const auto p = ps::plan_pass<DlSPhi, kTDlSPhi>(in.n_trg, in.n_src, resident[6]);
            e = ps::run_pass<DlSPhi, kTDlSPhi, kWDlSPhi>(a, p, ws, stream, none);
        }
    }
    return e;
}

}  // namespace stokes
