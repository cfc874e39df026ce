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
    if (a.accumulate) {
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
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&g)[NT],
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
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&q)[NT],
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
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&v)[NT],
                                bool skip, double (&acc)[NACC]) {
        const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
        const double r2 = dot3(dx, dy, dz, dx, dy, dz);
        const double ri = ri_of<M>(r2, skip);
        const double ri2 = ri * ri, ri3 = ri2 * ri;
        const double rqm = dot3(dx, dy, dz, s.qx, s.qy, s.qz);
        const double rgm = dot3(dx, dy, dz, s.gx, s.gy, s.gz);
        const double rgp = dot3(dx, dy, dz, v[0], v[1], v[2]);
        const double rqp = dot3(dx, dy, dz, v[3], v[4], v[5]);
        const double ab = dot3(v[0], v[1], v[2], s.qx, s.qy, s.qz) + dot3(v[3], v[4], v[5], s.gx, s.gy, s.gz);
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
    template <bool M>
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&g)[NT],
                                bool skip, double (&acc)[NACC]) {
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
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&v)[NT],
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
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&)[NT],
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
    __device__ static void pair(const Rec& s, double x, double y, double z, const double (&nv)[NT],
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

// launch shapes (targets per lane, minimum waves per SIMD)
constexpr int kTSlT = 4, kWSlT = 3;
constexpr int kTSlS = 2, kWSlS = 4;
constexpr int kTSym = 2, kWSym = 3;
constexpr int kTDlT = 4, kWDlT = 3;
constexpr int kTDlS = 2, kWDlS = 3;
constexpr int kTSlSF = 4, kWSlSF = 4;
constexpr int kTDlSPhi = 4, kWDlSPhi = 4;

}  // namespace

void vjp_resident(int n_cu, int out[kVjpPasses]) {
    out[0] = ps::resident_blocks<SlT, kTSlT, kWSlT>(n_cu);
    out[1] = ps::resident_blocks<SlS, kTSlS, kWSlS>(n_cu);
    out[2] = ps::resident_blocks<SlSym, kTSym, kWSym>(n_cu);
    out[3] = ps::resident_blocks<DlT, kTDlT, kWDlT>(n_cu);
    out[4] = ps::resident_blocks<DlS, kTDlS, kWDlS>(n_cu);
    out[5] = ps::resident_blocks<SlSF, kTSlSF, kWSlSF>(n_cu);
    out[6] = ps::resident_blocks<DlSPhi, kTDlSPhi, kWDlSPhi>(n_cu);
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

hipError_t launch_dl_vjp(const VjpInputs& in, const int resident[kVjpPasses], void* ws,
                         hipStream_t stream) {
    hipError_t e = hipSuccess;
    const KernelTimer none{};
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
