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
 * floating-point atomics, so a repeated call gives the same bits.
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
#define STOKES_OP_P2P_SL_VJP 6
#define STOKES_OP_P2P_DL_VJP 7

/* Largest point count per side accepted by any call. */
#define STOKES_MAX_POINTS ((int64_t)1 << 30)

typedef struct stokes_ctx stokes_ctx;            /* opaque, one per device */
typedef struct stokes_p2p_plan stokes_p2p_plan;  /* opaque leaf layout on the device */
typedef struct stokes_fmm_plan stokes_fmm_plan;  /* opaque FMM operators on the device */

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

/* Each-pair-once evaluation of shared point sets (on by default).  When a
 * single-layer call's sources are its targets (src_xyz == trg_xyz, n_src ==
 * n_trg, and with the same-group rule one array for both groups) and its
 * workspace holds what stokes_workspace_size reports for n_src == n_trg, the
 * Stokeslet's symmetry S(x, y) = S(y, x) lets every unordered pair be
 * evaluated once for both of its points (float64).  on = 0 makes such calls
 * evaluate each ordered pair separately, as for distinct point sets (tests,
 * benchmarks).  Results agree within the float64 bound either way.  Not
 * thread-safe against running calls. */
int stokes_set_pair_symmetry(stokes_ctx* ctx, int32_t on);

/* Test-only record of the mixed-precision split (float32 pairs, float64 near
 * pairs, excluded pairs; the near rule of stokes_exclusion). While an array
 * is registered, every STOKES_MIXED call of stokes_sl_eval, stokes_dl_eval,
 * stokes_sl_eval_noalloc, stokes_p2p_leaf_eval and stokes_p2p_plan_eval with
 * these n_trg and n_src runs instrumented copies of its kernels, which add,
 * for each (target t, source s) pair they take, one class code into
 * classes[t * n_src + s] (device memory, int32, zeroed by the caller):
 * STOKES_PAIR_F32, _F64 or _SKIP (same group, or zero distance). A pair
 * taken once holds exactly one code; a pair a leaf-to-leaf sum does not list
 * stays 0. The instrumented kernels are slow (one atomic add per pair).
 * classes = NULL unregisters; a mixed call of other sizes fails with
 * STOKES_EINVAL while one is registered. FP64 calls ignore it. */
#define STOKES_PAIR_F32 1
#define STOKES_PAIR_F64 (1 << 8)
#define STOKES_PAIR_SKIP (1 << 16)
int stokes_debug_pair_classes(stokes_ctx* ctx, int32_t* classes, int64_t n_trg, int64_t n_src);

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
 * and options needs.  For leaf-to-leaf ops n_leaves is the leaf count, and
 * for STOKES_OP_P2P_SL_VJP / _DL_VJP n_ulist the list length; others ignore
 * them.  May
 * be 0.  For STOKES_OP_SL with n_src == n_trg the size covers the
 * each-pair-once sum of a shared point set (its column partials grow as n^2:
 * about 0.9 GB for 278,528 points); a workspace of at least the size for
 * distinct point sets still works, one pair at a time. */
int stokes_workspace_size(const stokes_ctx* ctx, int32_t op, int64_t n_src, int64_t n_trg,
                          int32_t n_leaves, int64_t n_ulist, const stokes_opts* opts, size_t* bytes);

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

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): stokes_sl_eval with its scratch in a library-owned static
 * device array of STOKES_NOALLOC_SCRATCH_BYTES (64 MiB) instead of a caller
 * workspace.  Every GPU that the library runs on holds one such array for the
 * life of the process.  Arguments, results and errors otherwise as
 * stokes_sl_eval; every ordered pair is evaluated separately (the kernels
 * and launch shape of stokes_sl_eval with pair symmetry off, so bitwise its
 * values then), also on shared point sets.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine.  Sizes whose scratch (stokes_workspace_size with STOKES_OP_SL)
 * exceeds the array are rejected with STOKES_EWORKSPACE before any launch:
 * on a device with 256 compute units, about 230,000 sources and targets each
 * (a shared point set) in float64 and 300,000 in mixed precision.  All calls on one GPU share its array: two calls
 * whose executions overlap on that GPU (from other streams, threads or
 * contexts) race and may both return wrong results; order them on one
 * stream.  Nothing in the array needs to start at zero: every call writes all
 * of the scratch it reads. */
#define STOKES_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int stokes_sl_eval_noalloc(stokes_ctx* ctx, int64_t n_src, const double* src_xyz,
                           const double* density, const double* weight, int64_t n_trg,
                           const double* trg_xyz, double mu, const stokes_exclusion* excl,
                           const stokes_opts* opts, double* vel_out, void* stream);

/* Double-layer sum (stresslet), after eq. (double_layer_int_eq):
 *   vel_out(3, n_trg) (=|+=) 6/(8 pi) sum_m' r (r.n_m)(r.q_m)/rho^5,
 *   q_m = weight_m * density_m, n_m = normal(:, m) (unit, outward).
 * The kernel has no viscosity.  Other arguments as stokes_sl_eval. */
int stokes_dl_eval(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                   const double* weight, const double* normal, int64_t n_trg,
                   const double* trg_xyz, const stokes_exclusion* excl, const stokes_opts* opts,
                   double* vel_out, void* workspace, size_t ws_bytes, void* stream);

/* ---- leaf-to-leaf (P2P) form of the FMM near field, Sec. 3.1 ------------- */

/* For each leaf L and each target x_n of L:
 *   vel_out(:, n) (=|+=) pref * sum over sources y_m of the leaves in U(L),
 *   minus the pair rule, of K(x_n - y_m) q_m,
 * with K the single layer (kernel = STOKES_KERNEL_SL, uses mu, normal may be
 * NULL) or the double layer (STOKES_KERNEL_DL, needs normal, ignores mu).
 * Leaf layout (DEVICE arrays, read during the call, caller-owned):
 * src_leaf_ofs and trg_leaf_ofs (n_leaves+1 int64 each) start at 0, never
 * decrease and end at n_src / n_trg; ulist_ofs (n_leaves+1 int64) starts at
 * 0, never decreases and ends at n_ulist; every ulist entry (int32) lies in
 * [0, n_leaves).  Leaf L owns sources [src_leaf_ofs[L], src_leaf_ofs[L+1])
 * and targets [trg_leaf_ofs[L], trg_leaf_ofs[L+1]); its targets sum over the
 * sources of leaves ulist[ulist_ofs[L] .. ulist_ofs[L+1]) (a leaf listed
 * twice is summed twice).  Point arrays are in leaf order.  The layout is
 * checked on the device, with no host round trip: if it breaks any rule
 * above, nothing outside the arrays is read and every component of vel_out
 * becomes NaN (also when accumulating); the call itself returns STOKES_OK.
 * The work items (64-target pieces of the leaves, largest first) are built
 * in the workspace on every call; stokes_workspace_size(STOKES_OP_P2P_*,
 * n_src, n_trg, n_leaves) sizes it.  Other arguments as stokes_sl_eval. */
int stokes_p2p_leaf_eval(stokes_ctx* ctx, int32_t kernel, int64_t n_src, const double* src_xyz,
                         const double* density, const double* weight, const double* normal, int64_t n_trg,
                         const double* trg_xyz, int32_t n_leaves, const int64_t* src_leaf_ofs,
                         const int64_t* trg_leaf_ofs, const int64_t* ulist_ofs, const int32_t* ulist,
                         int64_t n_ulist, double mu, const stokes_exclusion* excl, const stokes_opts* opts,
                         double* vel_out, void* workspace, size_t ws_bytes, void* stream);

/* The same sum with the layout prepared once from HOST arrays: the plan
 * validates them on the host (the rules above; a breach returns
 * STOKES_EINVAL and creates nothing), cuts and sorts the work items once and
 * owns their device copy until stokes_p2p_plan_destroy; it is read-only
 * afterwards.  For a layout that is evaluated many times. */
int stokes_p2p_plan_create(stokes_ctx* ctx, int32_t n_leaves, int64_t n_src, int64_t n_trg,
                           const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs,
                           const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist,
                           stokes_p2p_plan** plan);
void stokes_p2p_plan_destroy(stokes_p2p_plan* plan);
/* Pairs the plan visits (sum over leaves of targets x listed sources), before
 * the pair rule removes any. */
int stokes_p2p_plan_pairs(const stokes_p2p_plan* plan, int64_t* pairs);

/* stokes_p2p_leaf_eval on a plan's layout; n_src and n_trg must match the
 * plan.  Targets of no leaf are not written. */
int stokes_p2p_plan_eval(stokes_ctx* ctx, const stokes_p2p_plan* plan, int32_t kernel,
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
 * Outputs, precision and empty sets as stokes_sl_vjp.  On a shared point set
 * grad_src_xyz == grad_trg_xyz is allowed as there and receives the total
 * position gradient dL/dy + dL/dx: the target-side pass writes (or adds, when
 * accumulating) into it and the source-side pass adds to it.  When
 * grad_density and grad_trg_xyz are asked for without grad_src_xyz, one fused
 * pass over the pairs gives both; its grad_density adds per-target-block
 * partials in a fixed order (the workspace holds 3 doubles per source and
 * 1,024 targets). */
int stokes_dl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                  const double* weight, const double* normal, int64_t n_trg,
                  const double* trg_xyz, const stokes_exclusion* excl, const stokes_opts* opts,
                  const double* grad_vel, double* grad_density, double* grad_src_xyz,
                  double* grad_trg_xyz, void* workspace, size_t ws_bytes, void* stream);

/* Single-layer adjoint of stokes_p2p_leaf_eval (same inputs and device leaf
 * arrays, same rules for them): the sums of stokes_sl_vjp restricted to the
 * pairs the lists name (a pair listed k times counts k times), in float64.
 *   grad_trg_xyz: for target n of leaf L, c sum over the sources of L's list
 *                 of K(r_nm; g_n, q_m)  (one pass on the forward lists);
 *   grad_density, grad_src_xyz: for source m of leaf L', sums over the
 *                 targets of every leaf whose list holds L' (one pass each on
 *                 the transposed lists, built on the device by a stable sort
 *                 with no host round trip).
 * Targets of no leaf contribute nothing; sources listed by no leaf get zero.
 * Each output is optional (NULL skips it) and no two may overlap.  Malformed
 * leaf arrays make every component of the requested outputs NaN (also when
 * accumulating).  Deterministic: every sum runs in a fixed order.
 * Workspace: stokes_workspace_size(STOKES_OP_P2P_SL_VJP, n_src, n_trg,
 * n_leaves, n_ulist).  n_src == 0 or n_trg == 0 gives zero gradients (kept
 * when accumulating). */
int stokes_p2p_sl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                      const double* weight, int64_t n_trg, const double* trg_xyz, int32_t n_leaves,
                      const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs, const int64_t* ulist_ofs,
                      const int32_t* ulist, int64_t n_ulist, double mu, const stokes_exclusion* excl,
                      const stokes_opts* opts, const double* grad_vel, double* grad_density,
                      double* grad_src_xyz, double* grad_trg_xyz, void* workspace, size_t ws_bytes,
                      void* stream);

/* Double-layer adjoint of stokes_p2p_leaf_eval: the sums of stokes_dl_vjp
 * restricted to the listed pairs, in float64, with d = 6/(8 pi):
 *   grad_trg_xyz  (3,n_trg): d sum over listed m of G_nm  (forward lists);
 *   grad_density  (3,n_src): dL/dphi_m = d w_m sum over the targets n of the
 *                            leaves listing m's leaf of r (r.n_m)(r.g_n)/rho^5;
 *   grad_src_xyz  (3,n_src): -d sum over the same n of G_nm
 * (G as at stokes_dl_vjp; the source-side sums on the transposed lists).
 * Outputs, layout checks, NaN on malformed leaf arrays, determinism and empty
 * sets as stokes_p2p_sl_vjp.  Workspace: stokes_workspace_size(
 * STOKES_OP_P2P_DL_VJP, n_src, n_trg, n_leaves, n_ulist). */
int stokes_p2p_dl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                      const double* weight, const double* normal, int64_t n_trg, const double* trg_xyz,
                      int32_t n_leaves, const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs,
                      const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist,
                      const stokes_exclusion* excl, const stokes_opts* opts, const double* grad_vel,
                      double* grad_density, double* grad_src_xyz, double* grad_trg_xyz, void* workspace,
                      size_t ws_bytes, void* stream);

/* ---- check-point quadrature on and near a patched surface, Sec. 3.1 ------ */

/* A surface made of n_patches tensor-product patches, each given by q x q
 * nodes: node_xyz (3, n_patches*q*q), patch-major, node k = i*q + j of a patch
 * at parameters (u, v) = (nodes_1d[i], nodes_1d[j]) of [-1, 1]^2.  The patch is
 * the polynomial of degree q-1 in u and in v through its nodes, X_u x X_v must
 * point out of the surface, and (nodes_1d, weights_1d) is the 1-D rule of the
 * patch (Gauss-Legendre, Clenshaw-Curtis, ...) on [-1, 1].
 *   q           2 .. 24.
 *   eta         0 .. 3: the fine discretisation splits each patch into
 *               4^eta equal sub-squares, each with the same q x q rule.
 *   p           1 .. 15: p + 1 check points per target.
 *   R_frac      > 0: distance of the first check point from the surface, as
 *               a fraction of the patch size L (the square root of the area
 *               of the target's patch).
 *   r_frac      > 0: spacing of the check points, as a fraction of L.
 *   nodes_1d    HOST float64[q], strictly increasing, within [-1, 1].
 *   weights_1d  HOST float64[q], positive. */
typedef struct {
    int32_t       q;
    int32_t       eta;
    int32_t       p;
    double        R_frac;
    double        r_frac;
    const double* nodes_1d;
    const double* weights_1d;
} stokes_patch_rule;

/* The fine discretisation of Sec. 3.1 step 1 (the upsampling U), for every
 * patch: n_fine = n_patches * (2^eta q)^2 nodes, patch-major, fine node
 * I*(2^eta q) + J of a patch at (s_I, s_J), s_{a q + i} = -1 + (2a + 1 +
 * nodes_1d[i]) / 2^eta, the patch evaluated there.
 *   fine_xyz     (3, n_fine)  positions
 *   fine_density (3, n_fine)  U phi: the density interpolated like positions
 *   fine_weight  (n_fine)     weights_1d[i] weights_1d[j] / 4^eta |X_u x X_v|
 *   fine_normal  (3, n_fine)  X_u x X_v / |X_u x X_v|
 *   patch_size   (n_patches)  L = sqrt(sum of the patch's fine weights)
 * density (3, n_patches*q*q) may be NULL, and then fine_density is not
 * written.  R_frac, r_frac and p are not used.  Needs no workspace. */
int stokes_patch_upsample(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                          const double* node_xyz, const double* density, double* fine_xyz,
                          double* fine_density, double* fine_weight, double* fine_normal,
                          double* patch_size, void* stream);

/* Bytes of workspace stokes_dl_checkpoint_eval needs for these sizes. */
int stokes_checkpoint_workspace_size(const stokes_ctx* ctx, int64_t n_patches,
                                     const stokes_patch_rule* rule, int64_t n_trg,
                                     const stokes_opts* opts, size_t* bytes);

/* Double-layer velocity at targets on or near the surface by the check-point
 * quadrature of Sec. 3.1 (eqs. quad_check_points and sing-quad):
 *   1. fine discretisation and U phi, as stokes_patch_upsample;
 *   2. target t is the point x_t = y_t - d_t n_t, y_t = P(u_t, v_t) on patch
 *      trg_patch[t] with unit normal n_t = X_u x X_v / |X_u x X_v| there, and
 *      d_t >= 0 its distance inside (the closest-point search is the
 *      caller's: (u_t, v_t) is the closest point);
 *   3. check points c_ti = y_t - (R + i r) n_t, i = 0..p, R = R_frac L,
 *      r = r_frac L, L the size of patch trg_patch[t];
 *   4. u(c_ti): the double-layer sum of stokes_dl_eval (no pair rule) over
 *      the fine nodes;
 *   5. vel_out(:, t) (=|+=) sum_i e_i u(c_ti), e_i = prod_{k != i}
 *      (d_t - s_k)/(s_i - s_k), s_k = (R + k r) the check point distances.
 * The result is the limit from the side the check points lie on (inside a
 * closed surface): for a constant density it is -density, and on the
 * surface the principal value is the result plus density / 2.
 *   density     (3, n_patches*q*q) at the nodes.
 *   trg_patch   int32[n_trg], trg_uvd (3, n_trg) = rows u, v, d.  Both NULL:
 *               the targets are the n_patches*q*q nodes themselves, on the
 *               surface (n_trg must be that count); else both non-NULL.  A
 *               patch id outside [0, n_patches) gives NaN for that target.
 *   opts        precision of step 4 (STOKES_FP64 or STOKES_MIXED; the
 *               extrapolation amplifies its error by sum_i |e_i|, 511 for
 *               p = 8, R = r, d = 0) and accumulate for vel_out.
 *   check_xyz_out, check_vel_out  optional (3, n_trg*(p+1)) outputs, check
 *               point t*(p+1) + i: the check points and their velocities.
 * Every step runs on the GPU on `stream`; the workspace holds the fine
 * discretisation, the check points and the double-layer sum's scratch.
 * n_trg == 0 does nothing; n_patches == 0 needs n_trg == 0.  With timing on,
 * the double-layer sum is the timed kernel. */
int stokes_dl_checkpoint_eval(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                              const double* node_xyz, const double* density, int64_t n_trg,
                              const int32_t* trg_patch, const double* trg_uvd,
                              const stokes_opts* opts, double* vel_out, double* check_xyz_out,
                              double* check_vel_out, void* workspace, size_t ws_bytes,
                              void* stream);

/* ---- boundary integral equation on a closed patched surface, Sec. 2.1.2 -- */

/* The discretised interior Dirichlet problem of eq. (double_layer_int_eq) at
 * the patch nodes, eq. (int_eq_disc): find the double-layer density phi whose
 * velocity u = D phi inside the surface takes the values g on it,
 *   A phi = g,   A = L_in - N,
 *   L_in phi   the limit from inside of D phi at every node: the check-point
 *              quadrature of stokes_dl_checkpoint_eval with the nodes as
 *              on-surface targets (= (D_pv - I/2) phi for this kernel, which
 *              gives -phi for a constant phi);
 *   (N phi)_l  = n_l sum_m w_m n_m . phi_m, the rank-completing term, with the
 *              node normals and weights of the patch polynomial (the fine
 *              discretisation with eta = 0).
 * The paper writes (I/2 + D + N); with the sign of this kernel the interior
 * operator is D_pv - I/2, and -N keeps the eigenvalue that N moves (minus
 * the surface area) on the side of the others (-1 .. 0).  For compatible data
 * (sum of w g . n = 0) N phi vanishes at the solution.
 * The surface must be closed, with X_u x X_v pointing out of it.
 * phi, g and out are (3, N) with N = n_patches * q * q nodes in node order. */

/* Workspace of stokes_bie_apply (max_iter = 0) or of stokes_bie_solve with
 * that iteration cap. */
int stokes_bie_workspace_size(const stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                              int32_t max_iter, const stokes_opts* opts, size_t* bytes);

/* out (=|+=) A phi.  opts: precision of the double-layer sum, accumulate. */
int stokes_bie_apply(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                     const double* node_xyz, const double* phi, const stokes_opts* opts, double* out,
                     void* workspace, size_t ws_bytes, void* stream);

/* GMRES on A phi = g (Sec. 3.1, "Discretizing the integral equation"; the
 * paper caps it at 30 iterations): phi_0 = 0, no restart, Arnoldi with
 * classical Gram-Schmidt applied twice, Givens rotations.  Stops when the
 * residual estimate |g - A phi_k| / |g| is <= rtol, at max_iter (1..100)
 * iterations, or when the Krylov space becomes invariant.
 *   phi_out            (3, N) the solution (zeros when g == 0).
 *   iterations         host int32: iterations done.
 *   residual_history   host float64[max_iter + 1] or NULL: entries
 *                      0..iterations get the residual estimates (entry 0 = 1).
 * Every matrix-vector product and vector operation runs on the GPU on
 * `stream`; the host reads the Arnoldi coefficients back each iteration, so
 * the call blocks until the solve is done.  opts.accumulate must be 0.
 * Returns STOKES_EINVAL if g holds non-finite values.  FP64 results are
 * deterministic. */
int stokes_bie_solve(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                     const double* node_xyz, const double* g, int32_t max_iter, double rtol,
                     const stokes_opts* opts, double* phi_out, int32_t* iterations,
                     double* residual_history, void* workspace, size_t ws_bytes, void* stream);

/* ---- collision candidates by spatial hashing, Sec. 4 (steps a-c of Sec. 3.3) */

/* Space-time bounding boxes: for each mesh m, the smallest axis-aligned box
 * holding its points mesh_ofs[m] .. mesh_ofs[m+1]-1 at the start (x0) and the
 * end (x1, NULL for meshes that do not move, such as wall patches) of the
 * time step, moved out by inflate >= 0 on every side (the near-zone margin of
 * Sec. 3.3 step a; 0 for collision candidates).
 *   mesh_ofs   device int64[n_meshes + 1]; entries are clamped to
 *              [0, n_points], and a mesh with mesh_ofs[m+1] <= mesh_ofs[m] is
 *              empty: lo = +inf, hi = -inf (it takes part in no pair).
 *   x0, x1     (3, n_points).
 *   box_lo, box_hi (3, n_meshes) outputs.
 * A NaN coordinate makes the mesh's box NaN, which the search treats as
 * empty. */
int stokes_space_time_boxes(stokes_ctx* ctx, int32_t n_meshes, const int64_t* mesh_ofs, int64_t n_points,
                            const double* x0, const double* x1, double inflate, double* box_lo,
                            double* box_hi, void* stream);

/* Workspace of stokes_collision_candidates for n_boxes boxes and room for
 * max_entries (box, grid cell) entries (at most 2^31). */
int stokes_collision_workspace_size(const stokes_ctx* ctx, int32_t n_boxes, int64_t max_entries,
                                    size_t* bytes);

/* Candidate pairs: boxes that share a cell of the grid of spacing cell_size
 * (the paper takes the mean box diagonal) whose origin is the lowest corner of
 * the valid boxes.  A box covers the cells floor((lo - origin) / cell_size) ..
 * floor((hi - origin) / cell_size) on each axis (float64), which are the cells
 * the paper's volume samples hash to; a box with lo > hi on some axis (empty,
 * or NaN) covers none.  Every unordered pair (i, j), i < j, sharing a cell is
 * reported once: pairs_out (2, capacity) int32, device, row 0 = i, row 1 =
 * j, ordered by the Morton key of the pair's lowest shared cell, then i, then
 * j.  Only the first min(*n_pairs, capacity) pairs are written; *n_pairs
 * (host) gets the total, so a call with capacity 0 counts them.  *n_entries
 * (host, may be NULL) gets the number of (box, cell) entries.
 * Errors found on the GPU, after kernels have run (outputs untouched):
 *   STOKES_EWORKSPACE    more than max_entries entries (*n_entries says how many);
 *   STOKES_EUNSUPPORTED  a cell coordinate of 2^21 or more, or an infinite corner.
 * The call blocks until the pairs are written. */
int stokes_collision_candidates(stokes_ctx* ctx, int32_t n_boxes, const double* box_lo,
                                const double* box_hi, double cell_size, int64_t max_entries,
                                int32_t* pairs_out, int64_t capacity, int64_t* n_pairs,
                                int64_t* n_entries, void* workspace, size_t ws_bytes, void* stream);

/* ---- fast multipole method, single and double layer, Sec. 3.1 "Far evaluation" */

/* The paper evaluates the smooth quadrature for all targets at once with a
 * kernel-independent FMM (PVFMM, not described there).  This is the published
 * kernel-independent method on a uniform octree:
 *   tree      the cube (centre, half_width) split into 8^depth leaves; points
 *             outside it are counted in the nearest boundary leaf (and lose
 *             accuracy);
 *   surfaces  cube surfaces with `order` points per edge (6 (order-1)^2 + 2
 *             points) at 1.05 (upward equivalent, downward check) and 2.95
 *             (upward check, downward equivalent) box half-widths;
 *   passes    P2M, M2M, M2L over interaction lists, L2L, L2P, and the direct
 *             sum over the 27 leaves around each target's leaf (zero-distance
 *             pairs skipped).
 * Its error against the direct sum falls with `order` (single layer: about
 * 1e-3 at 4, 1e-4 at 6, 1e-6 at 8, 1e-7 at 10 on clustered points; double
 * layer up to ten times that below order 10); there is no pair rule (all
 * pairs, as in the paper, whose self-cell terms are handled by its singular
 * quadrature).
 * The plan holds the check-to-equivalent pseudo-inverses (singular values
 * below 1e-10 of the largest dropped), computed on the host at creation by a
 * threaded Jacobi SVD (about 0.1 s at order 4, 1.5 s at 6, 8 s at 8, 30 s at
 * 10 on 8 cores), and the M2L operators: for each of the 8 positions of a box
 * in its parent, its 189 interaction-list translations and the
 * parent-to-child one at unit scale, built on the device (8 x 190 x m^2
 * doubles, m = 3 (6 (order-1)^2 + 2) rounded up to 16: 0.4 GB at order 4,
 * 2.6 GB at 6, 9.8 GB at 8, 26 GB at 10).  All of it is device memory owned
 * by the plan until stokes_fmm_plan_destroy. */
int stokes_fmm_plan_create(stokes_ctx* ctx, int32_t order, stokes_fmm_plan** plan);   /* order 2..10 */
void stokes_fmm_plan_destroy(stokes_fmm_plan* plan);

/* Workspace for n_src sources, n_trg targets and depth (2..7): the per-box
 * densities grow as 8^depth * 6 * (6 (order-1)^2 + 2) doubles, the check
 * matrix of a level as 3 min(8^depth, max(n_src, n_trg)) + 262,656 columns of
 * m doubles (m as above), plus 32,768 columns of 3 (6 (order-1)^2 + 2) doubles
 * for the split pseudo-inverse products.  excl (may be NULL) as in the
 * evaluation: the same-group rule adds about 150 bytes per point and 32 per
 * group. */
int stokes_fmm_workspace_size(const stokes_ctx* ctx, const stokes_fmm_plan* plan, int64_t n_src,
                              int64_t n_trg, int32_t depth, const stokes_exclusion* excl, size_t* bytes);

/* vel_out(3, n_trg) (=|+=) the single-layer sum of stokes_sl_eval by the
 * FMM.  Pair rule: excl NULL or STOKES_EXCL_NONE sums every pair (rho = 0
 * skipped), as the paper's FMM does.  STOKES_EXCL_SAME_GROUP (Sec. 2.2, the
 * other cells only) needs n_groups > 0 and every id of src_group and
 * trg_group in [0, n_groups): after the FMM, each group's sum onto itself
 * (pairs of one group, rho > 0) is evaluated exactly in float64 by the
 * leaf-to-leaf kernel (points sorted by group inside the workspace, every
 * group a leaf listing itself) and subtracted, so the result is the sum over
 * pairs of different groups within the FMM's error.  An id outside
 * [0, n_groups) makes every component of vel_out NaN (checked on the device).
 * group_h and near_frac are not used.  centre: HOST double[3]; half_width > 0.
 * opts.precision:
 * STOKES_FP64, or STOKES_MIXED to run the near field's pairs in float32 as
 * the mixed leaf-to-leaf sum does (about 1e-7 relative, far below the FMM's
 * own error); every other pass stays float64.  The near field is the
 * leaf-to-leaf sum of stokes_p2p_leaf_eval over the uniform tree's 27-leaf
 * lists, built in the workspace.  Asynchronous on `stream`; the sources and
 * targets are sorted into leaf order inside the workspace and the result is
 * written in the caller's order.  FP64 results are deterministic. */
int stokes_fmm_sl_eval(stokes_ctx* ctx, const stokes_fmm_plan* plan, int64_t n_src,
                       const double* src_xyz, const double* density, const double* weight,
                       int64_t n_trg, const double* trg_xyz, double mu, const double* centre,
                       double half_width, int32_t depth, const stokes_exclusion* excl,
                       const stokes_opts* opts, double* vel_out, void* workspace, size_t ws_bytes,
                       void* stream);

/* vel_out(3, n_trg) (=|+=) the double-layer sum of stokes_dl_eval by the
 * same FMM: the double-layer kernel in P2M and in the near field.  A double-layer field has a net flux (the sum of n . q over the
 * sources) that single-layer equivalent densities cannot carry, so each box
 * also carries a point source of that flux at its centre (velocity
 * sigma r / (4 pi rho^3)); its equivalent density holds the flux-free rest.
 * Other arguments, the pair rule included, as stokes_fmm_sl_eval (no mu: the
 * kernel has none). */
int stokes_fmm_dl_eval(stokes_ctx* ctx, const stokes_fmm_plan* plan, int64_t n_src,
                       const double* src_xyz, const double* density, const double* weight,
                       const double* normal, int64_t n_trg, const double* trg_xyz,
                       const double* centre, double half_width, int32_t depth,
                       const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out,
                       void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STOKES_MI355X_H */
