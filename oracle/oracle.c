/*
 * Stokes kernel-sum ORACLE -- test infrastructure only.
 *
 * A plain, slow, FP64 CPU implementation of the sums that the HIP library
 * computes.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may call it; the product path never does.  It shares no code,
 * header or constant with the GPU library.
 *
 * What it computes (Lu, Morse, Rahimian, Stadler, Zorin, SC'19):
 *   - single-layer (Stokeslet) potential, eq. (sl_stokes) of Sec. 2.1.1:
 *       S(x,y) f = 1/(8 pi mu) * ( f/|r| + r (r.f)/|r|^3 ),  r = x - y
 *   - double-layer (stresslet) kernel, after eq. (double_layer_int_eq):
 *       D(x,y) phi = 6/(8 pi) * r (r.n(y)) (r.phi)/|r|^5,  n = source normal
 *   - the smooth N-body quadrature of eq.
 *     (smooth_double_layer_int_eq_patches_disc): the kernel times the
 *     quadrature weight w_l times the density at node l, summed over nodes;
 *     the same form is used for the single layer over cell surfaces.
 *   - the "other cells only" rule of the explicit step (Sec. 2.2, step 1(d):
 *     sum over j != i): a pair whose source and target carry the same group
 *     id is skipped when the same-group rule is on.  A pair at distance 0 is
 *     always skipped (reading of a case the paper leaves open).
 *   - the near-field (leaf-to-leaf) form of the FMM evaluation of Sec. 3.1
 *     ("Far evaluation"): each target leaf sums over the sources of the
 *     leaves in its interaction list only.
 *   - vector-Jacobian products of these sums, obtained by differentiating
 *     the definitions by hand (the paper has no gradients).
 *
 * Every sum runs over the sources in index order and accumulates each output
 * component with Neumaier's compensated summation, so the oracle's own error
 * stays near one rounding of the exact sum.  Arrays are structure-of-arrays:
 * a 3-vector field over N points is x[0..N), y[N..2N), z[2N..3N).
 *
 * Build: gcc -O3 -fopenmp -fPIC -shared (no -ffast-math, which would break
 * the compensated sums).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

#define ORACLE_PI 3.14159265358979323846

/* ---- compensated accumulation (Neumaier's variant of Kahan summation) ---- */
typedef struct { double s, c; } csum;

static inline void cadd(csum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static inline double cval(const csum* a) { return a->s + a->c; }

/* ---- pair rule: the same-group exclusion and the zero-distance rule ---- */
static inline int pair_skipped(int excl, const int32_t* gs, int64_t m,
                               const int32_t* gt, int64_t n, double r2)
{
    if (r2 == 0.0) return 1;
    if (excl == 1 && gs[m] == gt[n]) return 1;
    return 0;
}

/* ---- kernels applied to one pair ----------------------------------------
 * r = x - y.  These are the bare kernels without the 1/(8 pi mu) or 6/(8 pi)
 * prefactors, which the callers apply once to the finished sum.           */

/* Stokeslet: q/rho + r (r.q)/rho^3 */
static inline void sl_pair(const double r[3], const double q[3], double out[3])
{
    double r2 = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
    double rho = sqrt(r2);
    double rho3 = rho * r2;
    double rq = r[0]*q[0] + r[1]*q[1] + r[2]*q[2];
    for (int i = 0; i < 3; i++) out[i] = q[i] / rho + r[i] * rq / rho3;
}

/* Stresslet applied to (n, q): r (r.n)(r.q)/rho^5 */
static inline void dl_pair(const double r[3], const double nv[3], const double q[3], double out[3])
{
    double r2 = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
    double rho = sqrt(r2);
    double rho5 = r2 * r2 * rho;
    double rn = r[0]*nv[0] + r[1]*nv[1] + r[2]*nv[2];
    double rq = r[0]*q[0] + r[1]*q[1] + r[2]*q[2];
    for (int i = 0; i < 3; i++) out[i] = r[i] * rn * rq / rho5;
}

/* Gradient with respect to r of a . [S-kernel] b, i.e. of
 *   (a.b)/rho + (r.a)(r.b)/rho^3:
 *   K(r;a,b) = [ (r.b) a + (r.a) b - (a.b) r ]/rho^3 - 3 (r.a)(r.b) r/rho^5 */
static inline void sl_grad_pair(const double r[3], const double a[3], const double b[3], double out[3])
{
    double r2 = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
    double rho = sqrt(r2);
    double rho3 = rho * r2;
    double rho5 = rho3 * r2;
    double ra = r[0]*a[0] + r[1]*a[1] + r[2]*a[2];
    double rb = r[0]*b[0] + r[1]*b[1] + r[2]*b[2];
    double ab = a[0]*b[0] + a[1]*b[1] + a[2]*b[2];
    for (int i = 0; i < 3; i++)
        out[i] = (rb * a[i] + ra * b[i] - ab * r[i]) / rho3 - 3.0 * ra * rb * r[i] / rho5;
}

/* Gradient with respect to r of (r.n)(r.q)(r.g)/rho^5:
 *   [ (r.q)(r.g) n + (r.n)(r.g) q + (r.n)(r.q) g ]/rho^5 - 5 (r.n)(r.q)(r.g) r/rho^7 */
static inline void dl_grad_pair(const double r[3], const double nv[3], const double q[3],
                                const double g[3], double out[3])
{
    double r2 = r[0]*r[0] + r[1]*r[1] + r[2]*r[2];
    double rho = sqrt(r2);
    double rho5 = r2 * r2 * rho;
    double rho7 = rho5 * r2;
    double rn = r[0]*nv[0] + r[1]*nv[1] + r[2]*nv[2];
    double rq = r[0]*q[0] + r[1]*q[1] + r[2]*q[2];
    double rg = r[0]*g[0] + r[1]*g[1] + r[2]*g[2];
    for (int i = 0; i < 3; i++)
        out[i] = (rq * rg * nv[i] + rn * rg * q[i] + rn * rq * g[i]) / rho5
               - 5.0 * rn * rq * rg * r[i] / rho7;
}

static inline void load3(const double* a, int64_t n, int64_t i, double v[3])
{
    v[0] = a[i]; v[1] = a[n + i]; v[2] = a[2 * n + i];
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------------------
 * Direct sums.  Targets x (3,nt); sources y (3,ns) with density f (3,ns) and
 * quadrature weight w (ns); DL sources also carry the normal nrm (3,ns).
 * Group ids gs (ns) / gt (nt) are read only when excl == 1.  Output u (3,nt).
 * ------------------------------------------------------------------------- */
void oracle_sl(int64_t ns, const double* y, const double* f, const double* w,
               const int32_t* gs, int64_t nt, const double* x, const int32_t* gt,
               double mu, int excl, double* u)
{
    const double c = 1.0 / (8.0 * ORACLE_PI * mu);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t n = 0; n < nt; n++) {
        double xn[3]; load3(x, nt, n, xn);
        csum acc[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t m = 0; m < ns; m++) {
            double ym[3], fm[3], r[3], q[3], t[3];
            load3(y, ns, m, ym); load3(f, ns, m, fm);
            for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
            if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
            for (int i = 0; i < 3; i++) q[i] = w[m] * fm[i];
            sl_pair(r, q, t);
            for (int i = 0; i < 3; i++) cadd(&acc[i], t[i]);
        }
        for (int i = 0; i < 3; i++) u[i * nt + n] = c * cval(&acc[i]);
    }
}

void oracle_dl(int64_t ns, const double* y, const double* phi, const double* w,
               const double* nrm, const int32_t* gs, int64_t nt, const double* x,
               const int32_t* gt, int excl, double* u)
{
    const double d = 6.0 / (8.0 * ORACLE_PI);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t n = 0; n < nt; n++) {
        double xn[3]; load3(x, nt, n, xn);
        csum acc[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t m = 0; m < ns; m++) {
            double ym[3], pm[3], nm[3], r[3], q[3], t[3];
            load3(y, ns, m, ym); load3(phi, ns, m, pm); load3(nrm, ns, m, nm);
            for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
            if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
            for (int i = 0; i < 3; i++) q[i] = w[m] * pm[i];
            dl_pair(r, nm, q, t);
            for (int i = 0; i < 3; i++) cadd(&acc[i], t[i]);
        }
        for (int i = 0; i < 3; i++) u[i * nt + n] = d * cval(&acc[i]);
    }
}

/* ---------------------------------------------------------------------------
 * Leaf-to-leaf (P2P) form.  Sources and targets are grouped by leaf: leaf L
 * owns sources [src_ofs[L], src_ofs[L+1]) and targets [trg_ofs[L],
 * trg_ofs[L+1]); its interaction list is ulist[ulist_ofs[L] .. ulist_ofs[L+1]).
 * kernel 0 = single layer (mu used, nrm unused), 1 = double layer.
 * ------------------------------------------------------------------------- */
void oracle_p2p(int kernel, int64_t ns, const double* y, const double* f,
                const double* w, const double* nrm, const int32_t* gs,
                int64_t nt, const double* x, const int32_t* gt, int32_t n_leaves,
                const int64_t* src_ofs, const int64_t* trg_ofs,
                const int64_t* ulist_ofs, const int32_t* ulist,
                double mu, int excl, double* u)
{
    const double pref = kernel == 0 ? 1.0 / (8.0 * ORACLE_PI * mu) : 6.0 / (8.0 * ORACLE_PI);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t L = 0; L < n_leaves; L++) {
        for (int64_t n = trg_ofs[L]; n < trg_ofs[L + 1]; n++) {
            double xn[3]; load3(x, nt, n, xn);
            csum acc[3] = {{0, 0}, {0, 0}, {0, 0}};
            for (int64_t k = ulist_ofs[L]; k < ulist_ofs[L + 1]; k++) {
                int32_t Ls = ulist[k];
                for (int64_t m = src_ofs[Ls]; m < src_ofs[Ls + 1]; m++) {
                    double ym[3], fm[3], r[3], q[3], t[3];
                    load3(y, ns, m, ym); load3(f, ns, m, fm);
                    for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
                    if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
                    for (int i = 0; i < 3; i++) q[i] = w[m] * fm[i];
                    if (kernel == 0) {
                        sl_pair(r, q, t);
                    } else {
                        double nm[3]; load3(nrm, ns, m, nm);
                        dl_pair(r, nm, q, t);
                    }
                    for (int i = 0; i < 3; i++) cadd(&acc[i], t[i]);
                }
            }
            for (int i = 0; i < 3; i++) u[i * nt + n] = pref * cval(&acc[i]);
        }
    }
}

/* ---------------------------------------------------------------------------
 * Vector-Jacobian products.  g (3,nt) is dL/du for a scalar loss L.  Each
 * output pointer may be NULL, which skips that output.  Weights and normals
 * are treated as constants (no derivative through the surface geometry).
 *
 * Single layer, with c = 1/(8 pi mu) and q_m = w_m f_m:
 *   dL/df_m = c w_m  sum_n S(r_nm) g_n           (S is symmetric and even)
 *   dL/dy_m = -c     sum_n K(r_nm; g_n, q_m)
 *   dL/dx_n =  c     sum_m K(r_nm; g_n, q_m)
 * ------------------------------------------------------------------------- */
void oracle_sl_vjp(int64_t ns, const double* y, const double* f, const double* w,
                   const int32_t* gs, int64_t nt, const double* x, const int32_t* gt,
                   double mu, int excl, const double* g,
                   double* grad_f, double* grad_y, double* grad_x)
{
    const double c = 1.0 / (8.0 * ORACLE_PI * mu);
    if (grad_f || grad_y) {
        #pragma omp parallel for schedule(dynamic, 8)
        for (int64_t m = 0; m < ns; m++) {
            double ym[3], fm[3], q[3];
            load3(y, ns, m, ym); load3(f, ns, m, fm);
            for (int i = 0; i < 3; i++) q[i] = w[m] * fm[i];
            csum af[3] = {{0, 0}, {0, 0}, {0, 0}}, ay[3] = {{0, 0}, {0, 0}, {0, 0}};
            for (int64_t n = 0; n < nt; n++) {
                double xn[3], gn[3], r[3], t[3];
                load3(x, nt, n, xn); load3(g, nt, n, gn);
                for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
                if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
                sl_pair(r, gn, t);
                for (int i = 0; i < 3; i++) cadd(&af[i], t[i]);
                sl_grad_pair(r, gn, q, t);
                for (int i = 0; i < 3; i++) cadd(&ay[i], t[i]);
            }
            for (int i = 0; i < 3; i++) {
                if (grad_f) grad_f[i * ns + m] = c * w[m] * cval(&af[i]);
                if (grad_y) grad_y[i * ns + m] = -c * cval(&ay[i]);
            }
        }
    }
    if (grad_x) {
        #pragma omp parallel for schedule(dynamic, 8)
        for (int64_t n = 0; n < nt; n++) {
            double xn[3], gn[3];
            load3(x, nt, n, xn); load3(g, nt, n, gn);
            csum ax[3] = {{0, 0}, {0, 0}, {0, 0}};
            for (int64_t m = 0; m < ns; m++) {
                double ym[3], fm[3], r[3], q[3], t[3];
                load3(y, ns, m, ym); load3(f, ns, m, fm);
                for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
                if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
                for (int i = 0; i < 3; i++) q[i] = w[m] * fm[i];
                sl_grad_pair(r, gn, q, t);
                for (int i = 0; i < 3; i++) cadd(&ax[i], t[i]);
            }
            for (int i = 0; i < 3; i++) grad_x[i * nt + n] = c * cval(&ax[i]);
        }
    }
}

/* Double layer, with d = 6/(8 pi) and q_m = w_m phi_m:
 *   dL/dphi_m = d w_m sum_n r (r.n_m)(r.g_n)/rho^5
 *   dL/dy_m   = -d    sum_n grad_r[(r.n_m)(r.q_m)(r.g_n)/rho^5]
 *   dL/dx_n   =  d    sum_m grad_r[(r.n_m)(r.q_m)(r.g_n)/rho^5]           */
void oracle_dl_vjp(int64_t ns, const double* y, const double* phi, const double* w,
                   const double* nrm, const int32_t* gs, int64_t nt, const double* x,
                   const int32_t* gt, int excl, const double* g,
                   double* grad_phi, double* grad_y, double* grad_x)
{
    const double d = 6.0 / (8.0 * ORACLE_PI);
    if (grad_phi || grad_y) {
        #pragma omp parallel for schedule(dynamic, 8)
        for (int64_t m = 0; m < ns; m++) {
            double ym[3], pm[3], nm[3], q[3];
            load3(y, ns, m, ym); load3(phi, ns, m, pm); load3(nrm, ns, m, nm);
            for (int i = 0; i < 3; i++) q[i] = w[m] * pm[i];
            csum ap[3] = {{0, 0}, {0, 0}, {0, 0}}, ay[3] = {{0, 0}, {0, 0}, {0, 0}};
            for (int64_t n = 0; n < nt; n++) {
                double xn[3], gn[3], r[3], t[3];
                load3(x, nt, n, xn); load3(g, nt, n, gn);
                for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
                if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
                dl_pair(r, nm, gn, t);
                for (int i = 0; i < 3; i++) cadd(&ap[i], t[i]);
                dl_grad_pair(r, nm, q, gn, t);
                for (int i = 0; i < 3; i++) cadd(&ay[i], t[i]);
            }
            for (int i = 0; i < 3; i++) {
                if (grad_phi) grad_phi[i * ns + m] = d * w[m] * cval(&ap[i]);
                if (grad_y) grad_y[i * ns + m] = -d * cval(&ay[i]);
            }
        }
    }
    if (grad_x) {
        #pragma omp parallel for schedule(dynamic, 8)
        for (int64_t n = 0; n < nt; n++) {
            double xn[3], gn[3];
            load3(x, nt, n, xn); load3(g, nt, n, gn);
            csum ax[3] = {{0, 0}, {0, 0}, {0, 0}};
            for (int64_t m = 0; m < ns; m++) {
                double ym[3], pm[3], nm[3], r[3], q[3], t[3];
                load3(y, ns, m, ym); load3(phi, ns, m, pm); load3(nrm, ns, m, nm);
                for (int i = 0; i < 3; i++) r[i] = xn[i] - ym[i];
                if (pair_skipped(excl, gs, m, gt, n, r[0]*r[0] + r[1]*r[1] + r[2]*r[2])) continue;
                for (int i = 0; i < 3; i++) q[i] = w[m] * pm[i];
                dl_grad_pair(r, nm, q, gn, t);
                for (int i = 0; i < 3; i++) cadd(&ax[i], t[i]);
            }
            for (int i = 0; i < 3; i++) grad_x[i * nt + n] = d * cval(&ax[i]);
        }
    }
}
