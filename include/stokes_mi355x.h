/*
 * stokes_mi355x.h -- C ABI of the MI355X (gfx950) Stokes kernel-sum library.
 *
 * The library sums the two Stokes kernels of the boundary-integral red-blood-
 * cell flow method of Lu, Morse, Rahimian, Stadler and Zorin (SC'19):
 *
 *   single layer (Stokeslet), eq. (sl_stokes), Sec. 2.1.1:
 *     u(x_n) = 1/(8 pi mu) sum_m' [ q_m/rho + r (r.q_m)/rho^3 ]
 *   double layer (stresslet), stated after eq. (double_layer_int_eq):
 *     u(x_n) = 6/(8 pi)    sum_m' r (r.n_m)(r.q_m)/rho^5
 *
 * with r = x_n - y_m (target minus source), rho = |r|, n_m the outward unit
 * normal at the source, and q_m = w_m f_m the density times the quadrature
 * weight (the smooth N-body quadrature of eq.
 * (smooth_double_layer_int_eq_patches_disc)).  sum_m' skips
 *   - pairs whose source and target carry the same group id when the
 *     same-group rule is on: the "other cells only" sum of the explicit time
 *     step (Sec. 2.2, step 1(d), j != i);
 *   - pairs at distance 0 (always).
 *
 * Layout.  Every 3-vector field over N points is structure-of-arrays float64:
 * x[0..N), y[N..2N), z[2N..3N), contiguous (a (3, N) row-major array).
 * Scalars per point (weights) are float64[N]; group ids are int32[N].
 *
 * Memory.  Unless a comment says "host", every array pointer is device
 * memory on the context's GPU, owned by the caller.  The library allocates
 * no user-visible memory during an evaluation: scratch comes from the
 * caller's workspace, whose size stokes_workspace_size() reports (the
 * workspace must be 256-byte aligned).  Outputs must not overlap any input.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the device's null stream).
 * Evaluations are asynchronous on it; the context is read-only after
 * creation, so calls with distinct outputs and workspaces may run
 * concurrently.  FP64 results are deterministic: fixed summation order, no
 * floating-point atomics.  One exception: grad_density of stokes_dl_vjp
 * when it comes from the fused pass (see there) is summed across target
 * blocks with float64 atomic adds, so it may differ in the last bits from
 * run to run.
 *
 * Errors.  Every call returns a status code.  Arguments are validated on the
 * host before anything is launched; a failed call launches nothing and
 * leaves outputs untouched.  stokes_last_error() returns a thread-local
 * message for the last non-OK status.  Faults inside a kernel surface at the
 * caller's next synchronisation with the stream.  The library never aborts.
 */
#ifndef STOKES_MI355X_H
#define STOKES_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define STOKES_OK            0
#define STOKES_EINVAL       (-1)  /* bad argument (null, size, alignment, enum, value, overlap) */
#define STOKES_EDEVICE      (-2)  /* no usable GPU, or a HIP runtime call failed */
#define STOKES_ELAUNCH      (-3)  /* a kernel launch was rejected */
#define STOKES_EWORKSPACE   (-4)  /* workspace missing, misaligned or too small */
#define STOKES_EUNSUPPORTED (-5)  /* device is not gfx950, or size beyond the supported range */

/* ---- enumerations -------------------------------------------------------- */
#define STOKES_FP64  0   /* every pair in float64 */
#define STOKES_MIXED 1   /* pairs in float32, near pairs and all sums in float64 */

#define STOKES_EXCL_NONE       0   /* only distance-0 pairs are skipped */
#define STOKES_EXCL_SAME_GROUP 1   /* also skip pairs with src_group == trg_group */

#define STOKES_KERNEL_SL 0
#define STOKES_KERNEL_DL 1

#define STOKES_OP_SL      0
#define STOKES_OP_DL      1
#define STOKES_OP_P2P_SL  2
#define STOKES_OP_P2P_DL  3
#define STOKES_OP_SL_VJP  4
#define STOKES_OP_DL_VJP  5

/* Largest point count per side accepted by any call. */
#define STOKES_MAX_POINTS ((int64_t)1 << 30)

typedef struct stokes_ctx stokes_ctx;            /* opaque, one per device */
typedef struct stokes_p2p_plan stokes_p2p_plan;  /* opaque leaf layout on the device */

/* Pair rule.
 *   mode       STOKES_EXCL_NONE or STOKES_EXCL_SAME_GROUP.
 *   src_group  int32[n_src]; required for SAME_GROUP, and in MIXED precision
 *              when group_h is given (it selects each source's spacing).
 *   trg_group  int32[n_trg]; required for SAME_GROUP.
 *   group_h    float64[n_groups] or NULL: mesh spacing h of each group (the
 *              square root of its area per point).  MIXED only.
 *   n_groups   length of group_h.
 *   near_frac  MIXED only: a pair whose float32 distance satisfies
 *              rho^2 <= (near_frac * h[src_group])^2 is evaluated in float64
 *              instead (a reading: the paper states no precision).  With
 *              group_h == NULL the radius is 0, so only coincident pairs
 *              take the float64 route (and contribute 0).  A source whose
 *              group id lies outside [0, n_groups) gets a NaN radius, which
 *              turns every output it touches into NaN.                    */
typedef struct {
    int32_t        mode;
    const int32_t* src_group;
    const int32_t* trg_group;
    const double*  group_h;
    int32_t        n_groups;
    double         near_frac;
} stokes_exclusion;

/* precision: STOKES_FP64 or STOKES_MIXED.
 * accumulate: 0 -> out = result; 1 -> out += result (superposition of
 *             several sums into one velocity, eq. (velocity_combined)). */
typedef struct {
    int32_t precision;
    int32_t accumulate;
} stokes_opts;

/* ---- context ------------------------------------------------------------- */

/* Binds device `device` (a HIP ordinal).  Fails with STOKES_EDEVICE if there
 * is no such device and STOKES_EUNSUPPORTED if it is not a gfx950.  Reads the
 * compute-unit count and clock used for launch shapes. */
int stokes_create(stokes_ctx** ctx, int device);
void stokes_destroy(stokes_ctx* ctx);

/* Thread-local description of the last failed call on this thread. */
const char* stokes_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int stokes_version(void);

/* Launch-shape override for tests: number of workgroups of the direct sums
 * (0 = automatic, the number resident on the device at once; at most 2^20).
 * Changes the work partition and the workspace size only; FP64 results stay
 * within the same error bound.  Not thread-safe against running calls. */
int stokes_set_grid_override(stokes_ctx* ctx, int32_t workgroups);

/* Kernel timing for benchmarks.  While enabled, every evaluation records a
 * pair of HIP events around its main summation kernel(s) (not the prep or
 * reduction kernels) on the call's stream.  stokes_timing_read waits for
 * those events, returns the summed milliseconds and the number of timed
 * launches since the last read (or since enabling), and starts a new count.
 * Enabling and reading are not thread-safe against concurrent evaluations
 * on the same context. */
int stokes_timing_enable(stokes_ctx* ctx, int on);
int stokes_timing_read(stokes_ctx* ctx, double* total_ms, int64_t* launches);

/* Bytes of workspace that a call of kind `op` (STOKES_OP_*) with these sizes
 * and options needs.  For P2P ops n_leaves is the plan's leaf count; for
 * others it is ignored.  May be 0. */
int stokes_workspace_size(const stokes_ctx* ctx, int32_t op, int64_t n_src, int64_t n_trg,
                          int32_t n_leaves, const stokes_opts* opts, size_t* bytes);

/* ---- direct sums ----------------------------------------------------------- */

/* Single-layer sum, eq. (sl_stokes) with the quadrature of eq.
 * (smooth_double_layer_int_eq_patches_disc):
 *   vel_out(3, n_trg) (=|+=) 1/(8 pi mu) sum_m' [q_m/rho + r (r.q_m)/rho^3],
 *   q_m = weight_m * density_m.
 * src_xyz (3,n_src), density (3,n_src), weight (n_src), trg_xyz (3,n_trg).
 * mu > 0 and finite.  excl may be NULL (= STOKES_EXCL_NONE, no near rule);
 * opts may be NULL (= FP64, overwrite).  n_src == 0 gives zeros (or leaves
 * vel_out unchanged when accumulating); n_trg == 0 does nothing. */
int stokes_sl_eval(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                   const double* weight, int64_t n_trg, const double* trg_xyz, double mu,
                   const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out,
                   void* workspace, size_t ws_bytes, void* stream);

/* Double-layer sum (stresslet), after eq. (double_layer_int_eq):
 *   vel_out(3, n_trg) (=|+=) 6/(8 pi) sum_m' r (r.n_m)(r.q_m)/rho^5,
 *   q_m = weight_m * density_m, n_m = normal(:, m) (unit, outward).
 * The kernel has no viscosity.  Other arguments as stokes_sl_eval. */
int stokes_dl_eval(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                   const double* weight, const double* normal, int64_t n_trg,
                   const double* trg_xyz, const stokes_exclusion* excl, const stokes_opts* opts,
                   double* vel_out, void* workspace, size_t ws_bytes, void* stream);

/* ---- leaf-to-leaf (P2P) form of the FMM near field, Sec. 3.1 ------------- */

/* Builds a leaf layout on the context's device from HOST arrays, validating
 * them: src_leaf_ofs and trg_leaf_ofs (n_leaves+1 int64 each) must start at
 * 0, be non-decreasing and end at n_src / n_trg; ulist_ofs (n_leaves+1) must
 * start at 0, be non-decreasing and end at n_ulist; every ulist entry (int32)
 * must lie in [0, n_leaves).  Leaf L owns sources [src_leaf_ofs[L],
 * src_leaf_ofs[L+1]) and targets [trg_leaf_ofs[L], trg_leaf_ofs[L+1]); its
 * targets sum over the sources of leaves ulist[ulist_ofs[L] .. ulist_ofs[L+1]).
 * A leaf listed twice is summed twice.  The plan owns device memory until
 * stokes_p2p_plan_destroy; it is read-only afterwards. */
int stokes_p2p_plan_create(stokes_ctx* ctx, int32_t n_leaves, int64_t n_src, int64_t n_trg,
                           const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs,
                           const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist,
                           stokes_p2p_plan** plan);
void stokes_p2p_plan_destroy(stokes_p2p_plan* plan);
/* Pairs the plan visits (sum over leaves of targets x listed sources), before
 * the pair rule removes any. */
int stokes_p2p_plan_pairs(const stokes_p2p_plan* plan, int64_t* pairs);

/* For each leaf L and each target x_n of L:
 *   vel_out(:, n) (=|+=) pref * sum over sources y_m of the leaves in U(L),
 *   minus the pair rule, of K(x_n - y_m) q_m,
 * with K the single layer (kernel = STOKES_KERNEL_SL, uses mu, normal may be
 * NULL) or the double layer (STOKES_KERNEL_DL, needs normal, ignores mu).
 * Point arrays are in the plan's leaf order; n_src and n_trg must match the
 * plan.  Targets of no leaf are not written. */
int stokes_p2p_leaf_eval(stokes_ctx* ctx, const stokes_p2p_plan* plan, int32_t kernel,
                         int64_t n_src, const double* src_xyz, const double* density,
                         const double* weight, const double* normal, int64_t n_trg,
                         const double* trg_xyz, double mu, const stokes_exclusion* excl,
                         const stokes_opts* opts, double* vel_out, void* workspace,
                         size_t ws_bytes, void* stream);

/* ---- vector-Jacobian products (hand-derived adjoints) --------------------- */

/* For a scalar loss L with grad_vel(3, n_trg) = dL/du of stokes_sl_eval
 * (same inputs), writes, each output optional (NULL skips it):
 *   grad_density (3,n_src): dL/df_m = c w_m sum_n' S(r_nm) g_n   (transposed sum)
 *   grad_src_xyz (3,n_src): dL/dy_m = -c sum_n' K(r_nm; g_n, q_m)
 *   grad_trg_xyz (3,n_trg): dL/dx_n =  c sum_m' K(r_nm; g_n, q_m)
 * with c = 1/(8 pi mu), g_n = grad_vel(:, n) and
 *   K(r;a,b) = [(r.b)a + (r.a)b - (a.b)r]/rho^3 - 3 (r.a)(r.b) r/rho^5,
 * the gradient in r of a.S(r)b.  Weights and normals are constants (no
 * derivative through the surface geometry).  The pair rule is the forward's.
 * Adjoint sums always run in float64 (opts->precision is ignored);
 * opts->accumulate adds into the outputs instead of overwriting them.
 * Shared point set: when src_xyz == trg_xyz, n_src == n_trg, the same-group
 * rule (if on) uses one group array, and grad_src_xyz == grad_trg_xyz (the
 * one array allowed to receive two gradients), that array receives the total
 * position gradient dL/dy + dL/dx and everything comes from one fused pass.
 * Otherwise the target-side and source-side gradients are separate passes.
 * n_src == 0 or n_trg == 0 gives zero gradients (kept when accumulating). */
int stokes_sl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                  const double* weight, int64_t n_trg, const double* trg_xyz, double mu,
                  const stokes_exclusion* excl, const stokes_opts* opts, const double* grad_vel,
                  double* grad_density, double* grad_src_xyz, double* grad_trg_xyz,
                  void* workspace, size_t ws_bytes, void* stream);

/* Double-layer adjoint, d = 6/(8 pi):
 *   grad_density (3,n_src): dL/dphi_m = d w_m sum_n' r (r.n_m)(r.g_n)/rho^5
 *   grad_src_xyz (3,n_src): dL/dy_m   = -d sum_n' G_nm
 *   grad_trg_xyz (3,n_trg): dL/dx_n   =  d sum_m' G_nm
 *   G = [(r.q)(r.g) n + (r.n)(r.g) q + (r.n)(r.q) g]/rho^5 - 5 (r.n)(r.q)(r.g) r/rho^7.
 * Outputs, precision and empty sets as stokes_sl_vjp.  When grad_density and
 * grad_trg_xyz are asked for without grad_src_xyz, one fused pass over the
 * pairs gives both; its grad_density is summed across target blocks with
 * float64 atomic adds (not bitwise reproducible from run to run). */
int stokes_dl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                  const double* weight, const double* normal, int64_t n_trg,
                  const double* trg_xyz, const stokes_exclusion* excl, const stokes_opts* opts,
                  const double* grad_vel, double* grad_density, double* grad_src_xyz,
                  double* grad_trg_xyz, void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STOKES_MI355X_H */
