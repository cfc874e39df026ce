// Host side of the C ABI declared in include/stokes_mi355x.h: argument
// validation, launch planning, workspace accounting and error reporting.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/stokes_mi355x.h"
#include "bie.hpp"
#include "checkpoint.hpp"
#include "common.hpp"
#include "fmm.hpp"
#include "groups.hpp"
#include "p2p.hpp"
#include "spatial.hpp"
#include "vjp.hpp"

struct stokes_ctx {
    int device;
    int n_cu;
    int clock_khz;
    int forced_grid;             // 0 = resident workgroup count
    int resident[2][2];          // [kernel][mixed]: resident workgroups of the direct sums
    int sym_resident[2];         // resident workgroups of the each-pair-once sums [forward, adjoint]
    bool pair_symmetry = true;   // shared point sets take the each-pair-once sum
    // test-only pair-class array of the mixed direct and leaf-to-leaf sums
    // (stokes_debug_pair_classes) and the sizes it was registered for
    int32_t* pair_class = nullptr;
    int64_t pair_class_trg = 0, pair_class_src = 0;
    int vjp_resident[stokes::kVjpPasses];   // resident workgroups of the adjoint pass kernels
    char arch[64];
    // device address of this device's copy of `scratch` (stokes_sl_eval_noalloc)
    void* scratch = nullptr;
    hipError_t scratch_status = hipErrorNotInitialized;
    // benchmark timing (see stokes_timing_enable)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;   // recorded, not yet read
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;    // reusable
};

namespace stokes {
// Event pair for the next timed launch on ctx (none when timing is off).
KernelTimer next_timer(stokes_ctx* ctx) {
    KernelTimer t;
    if (!ctx || !ctx->timing) return t;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (!ctx->spare.empty()) {
        ev = ctx->spare.back();
        ctx->spare.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
        return t;
    }
    ctx->events.push_back(ev);
    t.start = ev.first;
    t.stop = ev.second;
    return t;
}
}  // namespace stokes

// Scratch of stokes_sl_eval_noalloc, for callers that cannot allocate: the
// direct sum's workspace (packed source records, sub-tile summaries, partial
// sums, near-pass flags) lives here instead of in caller memory.  Each GPU that
// the library runs on holds its own copy until the process ends.  In host code
// this name is not a device address: stokes_create takes the address of the
// current device's copy with hipGetSymbolAddress and keeps it in the context,
// and only that address reaches kernels.
static __device__ __align__(256) unsigned char scratch[STOKES_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

const double kPi = 3.14159265358979323846;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Non-null (when count > 0) and naturally aligned.
bool arr_ok(const void* p, int64_t count, size_t align) {
    if (count <= 0) return true;
    return p != nullptr && aligned(p, align);
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Parsed {
    int precision = STOKES_FP64;
    int accumulate = 0;
    int excl = STOKES_EXCL_NONE;
    const int32_t* src_group = nullptr;
    const int32_t* trg_group = nullptr;
    const double* group_h = nullptr;
    int32_t n_groups = 0;
    double near_frac = 0.0;
};

int parse_common(const stokes_exclusion* ex, const stokes_opts* op, int64_t n_src, int64_t n_trg,
                 Parsed& p) {
    if (op) {
        if (op->precision != STOKES_FP64 && op->precision != STOKES_MIXED)
            return fail(STOKES_EINVAL, "opts.precision must be STOKES_FP64 or STOKES_MIXED");
        if (op->accumulate != 0 && op->accumulate != 1)
            return fail(STOKES_EINVAL, "opts.accumulate must be 0 or 1");
        p.precision = op->precision;
        p.accumulate = op->accumulate;
    }
    if (ex) {
        if (ex->mode != STOKES_EXCL_NONE && ex->mode != STOKES_EXCL_SAME_GROUP)
            return fail(STOKES_EINVAL, "exclusion.mode must be STOKES_EXCL_NONE or STOKES_EXCL_SAME_GROUP");
        p.excl = ex->mode;
        p.src_group = ex->src_group;
        p.trg_group = ex->trg_group;
        p.group_h = ex->group_h;
        p.n_groups = ex->n_groups;
        p.near_frac = ex->near_frac;
        if (p.excl == STOKES_EXCL_SAME_GROUP) {
            if (!arr_ok(p.src_group, n_src, 4) || (n_src > 0 && !p.src_group))
                return fail(STOKES_EINVAL, "same-group rule needs a 4-byte aligned src_group array");
            if (!arr_ok(p.trg_group, n_trg, 4) || (n_trg > 0 && !p.trg_group))
                return fail(STOKES_EINVAL, "same-group rule needs a 4-byte aligned trg_group array");
        }
        if (p.precision == STOKES_MIXED && p.group_h) {
            if (p.n_groups <= 0) return fail(STOKES_EINVAL, "group_h given with n_groups <= 0");
            if (!aligned(p.group_h, 8)) return fail(STOKES_EINVAL, "group_h must be 8-byte aligned");
            if (!(isfinite(p.near_frac) && p.near_frac >= 0.0))
                return fail(STOKES_EINVAL, "near_frac must be finite and >= 0");
            if (n_src > 0 && (!p.src_group || !aligned(p.src_group, 4)))
                return fail(STOKES_EINVAL, "the near rule needs a 4-byte aligned src_group array");
        }
        if (p.precision != STOKES_MIXED || !p.group_h) {
            p.group_h = nullptr;
            p.n_groups = 0;
        }
    }
    return STOKES_OK;
}

int check_sizes(int64_t n_src, int64_t n_trg) {
    if (n_src < 0 || n_trg < 0) return fail(STOKES_EINVAL, "point counts must be >= 0");
    if (n_src > STOKES_MAX_POINTS || n_trg > STOKES_MAX_POINTS)
        return fail(STOKES_EUNSUPPORTED, "point count above STOKES_MAX_POINTS");
    return STOKES_OK;
}

int check_workspace(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return STOKES_OK;
    if (!ws) return fail(STOKES_EWORKSPACE, "workspace is NULL but " + std::to_string(need) + " bytes are needed");
    if (!aligned(ws, 256)) return fail(STOKES_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(STOKES_EWORKSPACE, "workspace too small: " + std::to_string(ws_bytes) + " < " +
                                           std::to_string(need));
    return STOKES_OK;
}

int launch_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return STOKES_OK;
    return fail(STOKES_ELAUNCH, std::string(what) + ": " + hipGetErrorString(e));
}

stokes::SumInputs make_inputs(int kernel, const Parsed& p, int64_t n_src, const double* src_xyz,
                              const double* density, const double* weight, const double* normal,
                              int64_t n_trg, const double* trg_xyz, double pref) {
    stokes::SumInputs in{};
    in.kernel = kernel;
    in.mixed = p.precision == STOKES_MIXED;
    in.n_src = n_src;
    in.n_trg = n_trg;
    in.src_xyz = src_xyz;
    in.density = density;
    in.weight = weight;
    in.normal = normal;
    in.trg_xyz = trg_xyz;
    in.excl = p.excl;
    in.src_group = p.src_group;
    in.trg_group = p.trg_group;
    in.group_h = p.group_h;
    in.n_groups = p.n_groups;
    in.near_frac = p.near_frac;
    in.pref = pref;
    return in;
}

// Shared argument checks of the direct sums and their adjoints.
int check_points(int kernel, int64_t n_src, const double* src_xyz, const double* density,
                 const double* weight, const double* normal, int64_t n_trg, const double* trg_xyz) {
    if (!arr_ok(src_xyz, 3 * n_src, 8)) return fail(STOKES_EINVAL, "src_xyz must be non-NULL and 8-byte aligned");
    if (!arr_ok(density, 3 * n_src, 8)) return fail(STOKES_EINVAL, "density must be non-NULL and 8-byte aligned");
    if (!arr_ok(weight, n_src, 8)) return fail(STOKES_EINVAL, "weight must be non-NULL and 8-byte aligned");
    if (kernel == STOKES_KERNEL_DL && !arr_ok(normal, 3 * n_src, 8))
        return fail(STOKES_EINVAL, "normal must be non-NULL and 8-byte aligned");
    if (!arr_ok(trg_xyz, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "trg_xyz must be non-NULL and 8-byte aligned");
    return STOKES_OK;
}

// An output must not overlap any input array.
int check_no_alias(const void* out, size_t out_bytes, const char* name,
                   std::initializer_list<std::pair<const void*, size_t>> inputs) {
    for (const auto& in : inputs)
        if (overlaps(out, out_bytes, in.first, in.second))
            return fail(STOKES_EINVAL, std::string(name) + " overlaps an input array");
    return STOKES_OK;
}


// Check-point quadrature: the patch rule and the workspace layout.
int parse_patch_rule(const stokes_patch_rule* r, bool check_points, stokes::PatchRule& out) {
    if (!r) return fail(STOKES_EINVAL, "rule is NULL");
    if (r->q < 2 || r->q > stokes::kMaxQ)
        return fail(STOKES_EINVAL, "rule.q must be in [2, " + std::to_string(stokes::kMaxQ) + "]");
    if (r->eta < 0 || r->eta > stokes::kMaxEta)
        return fail(STOKES_EINVAL, "rule.eta must be in [0, " + std::to_string(stokes::kMaxEta) + "]");
    if (check_points) {
        if (r->p < 1 || r->p > stokes::kMaxP)
            return fail(STOKES_EINVAL, "rule.p must be in [1, " + std::to_string(stokes::kMaxP) + "]");
        if (!(isfinite(r->R_frac) && r->R_frac > 0.0) || !(isfinite(r->r_frac) && r->r_frac > 0.0))
            return fail(STOKES_EINVAL, "rule.R_frac and rule.r_frac must be finite and > 0");
    }
    if (!r->nodes_1d || !r->weights_1d)
        return fail(STOKES_EINVAL, "rule.nodes_1d and rule.weights_1d (host arrays of q) must be non-NULL");
    for (int k = 0; k < r->q; ++k) {
        const double t = r->nodes_1d[k], w = r->weights_1d[k];
        if (!(isfinite(t) && t >= -1.0 && t <= 1.0))
            return fail(STOKES_EINVAL, "rule.nodes_1d must lie within [-1, 1]");
        if (k > 0 && !(t > r->nodes_1d[k - 1]))
            return fail(STOKES_EINVAL, "rule.nodes_1d must be strictly increasing");
        if (!(isfinite(w) && w > 0.0)) return fail(STOKES_EINVAL, "rule.weights_1d must be finite and > 0");
    }
    out = stokes::PatchRule{};
    out.q = r->q;
    out.eta = r->eta;
    out.p = check_points ? r->p : 1;
    out.R = check_points ? r->R_frac : 0.0;
    out.r = check_points ? r->r_frac : 0.0;
    for (int k = 0; k < r->q; ++k) {
        out.t[k] = r->nodes_1d[k];
        out.w[k] = r->weights_1d[k];
    }
    return STOKES_OK;
}

struct CheckpointLayout {
    int64_t n_nodes = 0, n_fine = 0, n_check = 0;
    size_t off_fx = 0, off_fphi = 0, off_fw = 0, off_fn = 0, off_L = 0, off_cx = 0, off_cv = 0,
           off_direct = 0, total = 0;
    stokes::DirectPlan plan{};
};

// Point counts of the fine discretisation and the check points, checked
// against STOKES_MAX_POINTS, and (with_ws) the workspace regions.
int checkpoint_layout(const stokes_ctx* ctx, int64_t n_patches, const stokes::PatchRule& R, int64_t n_trg,
                      int mixed, bool with_ws, CheckpointLayout& lay) {
    if (n_patches < 0 || n_trg < 0) return fail(STOKES_EINVAL, "n_patches and n_trg must be >= 0");
    const int64_t qq = (int64_t)R.q * R.q, per_patch = qq << (2 * R.eta);
    if (n_patches > STOKES_MAX_POINTS / per_patch)
        return fail(STOKES_EUNSUPPORTED, "fine node count n_patches * (2^eta q)^2 above STOKES_MAX_POINTS");
    if (n_trg > STOKES_MAX_POINTS / (R.p + 1))
        return fail(STOKES_EUNSUPPORTED, "check point count n_trg * (p + 1) above STOKES_MAX_POINTS");
    lay.n_nodes = n_patches * qq;
    lay.n_fine = n_patches * per_patch;
    lay.n_check = n_trg * (R.p + 1);
    if (!with_ws || n_trg == 0 || n_patches == 0) return STOKES_OK;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = stokes::align_up(off + bytes, 256);
        return at;
    };
    const size_t f8 = (size_t)lay.n_fine * 8, c8 = (size_t)lay.n_check * 8;
    lay.off_fx = take(3 * f8);
    lay.off_fphi = take(3 * f8);
    lay.off_fw = take(f8);
    lay.off_fn = take(3 * f8);
    lay.off_L = take((size_t)n_patches * 8);
    lay.off_cx = take(3 * c8);
    lay.off_cv = take(3 * c8);
    lay.plan = stokes::plan_direct(1, mixed, lay.n_fine, lay.n_check, ctx->resident[1][mixed], ctx->forced_grid);
    lay.off_direct = off;
    lay.total = off + lay.plan.total;
    return STOKES_OK;
}

// Upsampling, check points, the double-layer sum at the check points and the
// extrapolation, on `st`, with the workspace regions of `lay` at `ws`.
hipError_t checkpoint_run(stokes_ctx* ctx, const stokes::PatchRule& R, const CheckpointLayout& lay,
                          int64_t n_patches, const double* node_xyz, const double* density, int64_t n_trg,
                          const int32_t* trg_patch, const double* trg_uvd, const Parsed& p, double* vel_out,
                          double* check_xyz_out, double* check_vel_out, char* ws, hipStream_t st) {
    double* fx = reinterpret_cast<double*>(ws + lay.off_fx);
    double* fphi = reinterpret_cast<double*>(ws + lay.off_fphi);
    double* fw = reinterpret_cast<double*>(ws + lay.off_fw);
    double* fn = reinterpret_cast<double*>(ws + lay.off_fn);
    double* L = reinterpret_cast<double*>(ws + lay.off_L);
    double* cx = check_xyz_out ? check_xyz_out : reinterpret_cast<double*>(ws + lay.off_cx);
    double* cv = check_vel_out ? check_vel_out : reinterpret_cast<double*>(ws + lay.off_cv);
    hipError_t e = stokes::launch_upsample(R, n_patches, node_xyz, density, fx, fphi, fw, fn, L, st);
    if (e == hipSuccess)
        e = stokes::launch_check_points(R, n_patches, node_xyz, L, n_trg, trg_patch, trg_uvd, cx, st);
    if (e == hipSuccess) {
        const stokes::SumInputs in = make_inputs(STOKES_KERNEL_DL, p, lay.n_fine, fx, fphi, fw, fn, lay.n_check,
                                                 cx, 6.0 / (8.0 * kPi));
        e = stokes::launch_direct(in, lay.plan, cv, 0, ws + lay.off_direct, st, stokes::next_timer(ctx));
    }
    if (e == hipSuccess)
        e = stokes::launch_extrapolate(R, n_patches, L, n_trg, trg_patch, trg_uvd, cv, vel_out, p.accumulate, st);
    return e;
}

// Boundary-integral operator (L_in - N) and its GMRES solve: workspace layout.
struct BieLayout {
    CheckpointLayout cp;
    int64_t n3 = 0;               // 3 * nodes
    size_t off_cp = 0, off_nn = 0, off_nw = 0, off_wn = 0, off_gx = 0, off_gL = 0, off_part = 0, off_dots = 0,
           off_coef = 0, off_V = 0, off_w = 0, total = 0;
};

int bie_layout(const stokes_ctx* ctx, int64_t n_patches, const stokes::PatchRule& R, int32_t max_iter, int mixed,
               BieLayout& lay) {
    if (max_iter < 0 || max_iter > stokes::kMaxKrylov)
        return fail(STOKES_EINVAL, "max_iter must be in [0, " + std::to_string(stokes::kMaxKrylov) + "]");
    if (n_patches < 0) return fail(STOKES_EINVAL, "n_patches must be >= 0");
    const int64_t qq = (int64_t)R.q * R.q;
    if (n_patches > STOKES_MAX_POINTS / qq) return fail(STOKES_EUNSUPPORTED, "node count above STOKES_MAX_POINTS");
    const int64_t nn = n_patches * qq;
    int rc = checkpoint_layout(ctx, n_patches, R, nn, mixed, true, lay.cp);
    if (rc) return rc;
    lay.n3 = 3 * nn;
    if (nn == 0) return STOKES_OK;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = stokes::align_up(off + bytes, 256);
        return at;
    };
    const size_t v8 = (size_t)lay.n3 * 8;
    lay.off_cp = take(lay.cp.total);
    lay.off_nn = take(v8);
    lay.off_nw = take((size_t)nn * 8);
    lay.off_wn = take(v8);
    lay.off_gx = take(v8);
    lay.off_gL = take((size_t)n_patches * 8);
    lay.off_part = take((size_t)(stokes::kMaxKrylov + 1) * stokes::reduce_blocks(lay.n3) * 8);
    lay.off_dots = take((size_t)(2 * stokes::kMaxKrylov + 4) * 8);
    lay.off_coef = take((size_t)(stokes::kMaxKrylov + 1) * 8);
    lay.off_V = take((size_t)(max_iter + 1) * v8);
    lay.off_w = take(v8);
    lay.total = off;
    return STOKES_OK;
}

// Node normals and weights of the patch polynomial (the fine discretisation
// with eta = 0), and w*n for the rank-completing term.
hipError_t bie_geometry(const stokes::PatchRule& R, const BieLayout& lay, int64_t n_patches, const double* node_xyz,
                        char* ws, hipStream_t st) {
    stokes::PatchRule R0 = R;
    R0.eta = 0;
    double* nn = reinterpret_cast<double*>(ws + lay.off_nn);
    double* nw = reinterpret_cast<double*>(ws + lay.off_nw);
    hipError_t e = stokes::launch_upsample(R0, n_patches, node_xyz, nullptr, reinterpret_cast<double*>(ws + lay.off_gx),
                                           nullptr, nw, nn, reinterpret_cast<double*>(ws + lay.off_gL), st);
    if (e != hipSuccess) return e;
    return stokes::launch_weighted_normals(reinterpret_cast<double*>(ws + lay.off_wn), nn, nw, lay.n3 / 3, st);
}

// out (=|+=) (L_in - N) phi; needs bie_geometry first.  dot_slot: where in the
// dots buffer n . phi lands.
hipError_t bie_apply_run(stokes_ctx* ctx, const stokes::PatchRule& R, const BieLayout& lay, int64_t n_patches,
                         const double* node_xyz, const double* phi, const Parsed& p, double* out, char* ws,
                         int dot_slot, hipStream_t st) {
    hipError_t e = checkpoint_run(ctx, R, lay.cp, n_patches, node_xyz, phi, lay.n3 / 3, nullptr, nullptr, p, out,
                                  nullptr, nullptr, ws + lay.off_cp, st);
    double* dots = reinterpret_cast<double*>(ws + lay.off_dots) + dot_slot;
    if (e == hipSuccess)
        e = stokes::launch_multi_dot(reinterpret_cast<const double*>(ws + lay.off_wn), lay.n3, 1, phi, lay.n3,
                                     reinterpret_cast<double*>(ws + lay.off_part), dots, st);
    if (e == hipSuccess)
        e = stokes::launch_combo_sub(out, reinterpret_cast<const double*>(ws + lay.off_nn), lay.n3, 1, dots, lay.n3,
                                     st);
    return e;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char* stokes_last_error(void) { return g_err.c_str(); }

int stokes_version(void) { return 1 * 10000 + 0 * 100 + 0; }

int stokes_create(stokes_ctx** ctx, int device) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0)
        return fail(STOKES_EDEVICE, std::string("no HIP device available: ") + hipGetErrorString(e));
    if (device < 0 || device >= count)
        return fail(STOKES_EDEVICE, "device ordinal " + std::to_string(device) + " out of range");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return fail(STOKES_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(STOKES_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
    stokes_ctx* c = new (std::nothrow) stokes_ctx{};
    if (!c) return fail(STOKES_EDEVICE, "out of host memory");
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->clock_khz = prop.clockRate;
    c->forced_grid = 0;
    strncpy(c->arch, prop.gcnArchName, sizeof(c->arch) - 1);
    {
        DeviceGuard dg(device);
        if (!dg.ok) {
            delete c;
            return fail(STOKES_EDEVICE, "cannot select the device");
        }
        for (int k = 0; k < 2; ++k)
            for (int m = 0; m < 2; ++m) c->resident[k][m] = stokes::direct_blocks_per_cu(k, m) * c->n_cu;
        stokes::vjp_resident(c->n_cu, c->vjp_resident);
        for (int v = 0; v < 2; ++v) c->sym_resident[v] = stokes::sym_blocks_per_cu(v) * c->n_cu;
        // this device's copy of the no-allocation scratch array (a failure
        // only disables stokes_sl_eval_noalloc, which reports it)
        void* sp = nullptr;
        c->scratch_status = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        c->scratch = c->scratch_status == hipSuccess ? sp : nullptr;
    }
    *ctx = c;
    return STOKES_OK;
}

void stokes_destroy(stokes_ctx* ctx) {
    if (!ctx) return;
    for (auto* v : {&ctx->events, &ctx->spare})
        for (auto& ev : *v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    delete ctx;
}

int stokes_timing_enable(stokes_ctx* ctx, int on) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    ctx->timing = on != 0;
    // event pairs made here, not inside timed evaluations
    while (ctx->timing && ctx->spare.size() + ctx->events.size() < 64) {
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (hipEventCreate(&ev.first) != hipSuccess) break;
        if (hipEventCreate(&ev.second) != hipSuccess) {
            (void)hipEventDestroy(ev.first);
            break;
        }
        ctx->spare.push_back(ev);
    }
    return STOKES_OK;
}

int stokes_timing_read(stokes_ctx* ctx, double* total_ms, int64_t* launches) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!total_ms || !launches) return fail(STOKES_EINVAL, "output pointer is NULL");
    double sum = 0.0;
    int64_t n = 0;
    for (auto& ev : ctx->events) {
        if (hipEventSynchronize(ev.second) != hipSuccess)
            return fail(STOKES_EDEVICE, "hipEventSynchronize failed while reading timings");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess)
            return fail(STOKES_EDEVICE, "hipEventElapsedTime failed while reading timings");
        sum += ms;
        ++n;
        ctx->spare.push_back(ev);
    }
    ctx->events.clear();
    *total_ms = sum;
    *launches = n;
    return STOKES_OK;
}

int stokes_set_grid_override(stokes_ctx* ctx, int32_t workgroups) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (workgroups < 0 || workgroups > (1 << 20))
        return fail(STOKES_EINVAL, "workgroups must be in [0, 2^20]");
    ctx->forced_grid = workgroups;
    return STOKES_OK;
}

int stokes_set_pair_symmetry(stokes_ctx* ctx, int32_t on) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (on != 0 && on != 1) return fail(STOKES_EINVAL, "on must be 0 or 1");
    ctx->pair_symmetry = on != 0;
    return STOKES_OK;
}

int stokes_debug_pair_classes(stokes_ctx* ctx, int32_t* classes, int64_t n_trg, int64_t n_src) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!classes) {
        ctx->pair_class = nullptr;
        ctx->pair_class_trg = ctx->pair_class_src = 0;
        return STOKES_OK;
    }
    if (n_trg <= 0 || n_src <= 0 || n_trg > (int64_t(1) << 40) / n_src)
        return fail(STOKES_EINVAL, "n_trg and n_src must be > 0 with n_trg * n_src <= 2^40");
    if (reinterpret_cast<uintptr_t>(classes) % 4 != 0) return fail(STOKES_EINVAL, "classes must be 4-byte aligned");
    ctx->pair_class = classes;
    ctx->pair_class_trg = n_trg;
    ctx->pair_class_src = n_src;
    return STOKES_OK;
}

// The pair-class array for a mixed call of these sizes (null when none is
// registered); a registered array of other sizes is an error.
static int pair_class_for(const stokes_ctx* ctx, int mixed, int64_t n_src, int64_t n_trg, int32_t** out) {
    *out = nullptr;
    if (!mixed || !ctx->pair_class) return STOKES_OK;
    if (n_trg != ctx->pair_class_trg || n_src != ctx->pair_class_src)
        return fail(STOKES_EINVAL, "the pair-class array was registered for other sizes");
    *out = ctx->pair_class;
    return STOKES_OK;
}

// Whether the single-layer sum with these sizes and precision has an
// each-pair-once form (used only when the call's point set is shared).
static bool sym_available(const stokes_ctx* ctx, int kernel, int mixed, int64_t n_src, int64_t n_trg) {
    return ctx->pair_symmetry && kernel == STOKES_KERNEL_SL && !mixed && n_src == n_trg && n_src > 0;
}

int stokes_workspace_size(const stokes_ctx* ctx, int32_t op, int64_t n_src, int64_t n_trg,
                          int32_t n_leaves, int64_t n_ulist, const stokes_opts* opts, size_t* bytes) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!bytes) return fail(STOKES_EINVAL, "bytes is NULL");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    Parsed p;
    rc = parse_common(nullptr, opts, n_src, n_trg, p);
    if (rc) return rc;
    const int mixed = p.precision == STOKES_MIXED;
    switch (op) {
        case STOKES_OP_SL:
        case STOKES_OP_DL: {
            if (n_src == 0 || n_trg == 0) { *bytes = 0; return STOKES_OK; }
            const int k = op == STOKES_OP_SL ? 0 : 1;
            *bytes = stokes::plan_direct(k, mixed, n_src, n_trg, ctx->resident[k][mixed],
                                         ctx->forced_grid).total;
            // equal sizes may be a shared point set: room for the each-pair-once sum
            if (sym_available(ctx, k, mixed, n_src, n_trg))
                *bytes = std::max(*bytes, stokes::plan_sym(0, n_src, ctx->sym_resident[0], ctx->forced_grid).total);
            return STOKES_OK;
        }
        case STOKES_OP_P2P_SL:
        case STOKES_OP_P2P_DL:
            if (n_leaves < 0) return fail(STOKES_EINVAL, "n_leaves must be >= 0");
            *bytes = stokes::p2p_workspace_bytes(op == STOKES_OP_P2P_SL ? 0 : 1, mixed, n_src, n_trg, n_leaves);
            return STOKES_OK;
        case STOKES_OP_P2P_SL_VJP:
        case STOKES_OP_P2P_DL_VJP:
            if (n_leaves < 0) return fail(STOKES_EINVAL, "n_leaves must be >= 0");
            if (n_ulist < 0) return fail(STOKES_EINVAL, "n_ulist must be >= 0");
            *bytes = stokes::p2p_vjp_workspace_bytes(op == STOKES_OP_P2P_SL_VJP ? 0 : 1, n_src, n_trg, n_leaves,
                                                     n_ulist);
            return STOKES_OK;
        case STOKES_OP_SL_VJP:
        case STOKES_OP_DL_VJP:
            *bytes = stokes::vjp_workspace_bytes(op == STOKES_OP_SL_VJP ? 0 : 1, n_src, n_trg,
                                                 ctx->vjp_resident);
            // equal sizes may be a shared point set: room for the each-pair-once adjoint
            if (op == STOKES_OP_SL_VJP && sym_available(ctx, STOKES_KERNEL_SL, 0, n_src, n_trg))
                *bytes = std::max(*bytes, stokes::plan_sym(1, n_src, ctx->sym_resident[1], ctx->forced_grid).total);
            return STOKES_OK;
        default:
            return fail(STOKES_EINVAL, "unknown op");
    }
}

static int direct_eval(stokes_ctx* ctx, int kernel, int64_t n_src, const double* src_xyz,
                       const double* density, const double* weight, const double* normal,
                       int64_t n_trg, const double* trg_xyz, double pref,
                       const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out,
                       void* workspace, size_t ws_bytes, void* stream, bool allow_sym = true) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    rc = check_points(kernel, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz);
    if (rc) return rc;
    if (!arr_ok(vel_out, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "vel_out must be non-NULL and 8-byte aligned");
    Parsed p;
    rc = parse_common(excl, opts, n_src, n_trg, p);
    if (rc) return rc;
    const size_t vb = (size_t)3 * n_trg * sizeof(double), sb = (size_t)3 * n_src * sizeof(double);
    rc = check_no_alias(vel_out, vb, "vel_out",
                        {{src_xyz, sb}, {density, sb}, {weight, (size_t)n_src * 8}, {normal, kernel ? sb : 0},
                         {trg_xyz, vb}, {workspace, ws_bytes}});
    if (rc) return rc;
    const int mixed = p.precision == STOKES_MIXED;
    stokes::DirectPlan plan{};
    size_t need = 0;
    if (n_src > 0 && n_trg > 0) {
        plan = stokes::plan_direct(kernel, mixed, n_src, n_trg, ctx->resident[kernel][mixed],
                                   ctx->forced_grid);
        need = plan.total;
    }
    rc = check_workspace(workspace, ws_bytes, need);
    if (rc) return rc;
    int32_t* pair_class = nullptr;
    if ((rc = pair_class_for(ctx, mixed, n_src, n_trg, &pair_class))) return rc;
    // a shared point set (one array, one group array) takes the each-pair-once
    // sum when the workspace has room for it
    const bool shared = src_xyz == trg_xyz && n_src == n_trg &&
                        (p.excl == STOKES_EXCL_NONE || p.src_group == p.trg_group);
    stokes::SymPlan splan{};
    bool use_sym = false;
    if (allow_sym && shared && sym_available(ctx, kernel, mixed, n_src, n_trg)) {
        splan = stokes::plan_sym(0, n_src, ctx->sym_resident[0], ctx->forced_grid);
        use_sym = ws_bytes >= splan.total;
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    stokes::SumInputs in = make_inputs(kernel, p, n_src, src_xyz, density, weight, normal,
                                       n_trg, trg_xyz, pref);
    in.pair_class = pair_class;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (use_sym)
        return launch_status(stokes::launch_sym(in, splan, vel_out, p.accumulate, workspace, st,
                                                stokes::next_timer(ctx)),
                             "stokes_sl_eval");
    return launch_status(stokes::launch_direct(in, plan, vel_out, p.accumulate, workspace, st,
                                               stokes::next_timer(ctx)),
                         kernel ? "stokes_dl_eval" : "stokes_sl_eval");
}

int stokes_sl_eval(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                   const double* weight, int64_t n_trg, const double* trg_xyz, double mu,
                   const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out,
                   void* workspace, size_t ws_bytes, void* stream) {
    if (!(isfinite(mu) && mu > 0.0)) return fail(STOKES_EINVAL, "mu must be finite and > 0");
    return direct_eval(ctx, STOKES_KERNEL_SL, n_src, src_xyz, density, weight, nullptr, n_trg,
                       trg_xyz, 1.0 / (8.0 * kPi * mu), excl, opts, vel_out, workspace, ws_bytes,
                       stream);
}

int stokes_sl_eval_noalloc(stokes_ctx* ctx, int64_t n_src, const double* src_xyz,
                           const double* density, const double* weight, int64_t n_trg,
                           const double* trg_xyz, double mu, const stokes_exclusion* excl,
                           const stokes_opts* opts, double* vel_out, void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!(isfinite(mu) && mu > 0.0)) return fail(STOKES_EINVAL, "mu must be finite and > 0");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    Parsed p;
    rc = parse_common(nullptr, opts, n_src, n_trg, p);
    if (rc) return rc;
    const int mixed = p.precision == STOKES_MIXED;
    size_t need = 0;
    if (n_src > 0 && n_trg > 0)
        need = stokes::plan_direct(STOKES_KERNEL_SL, mixed, n_src, n_trg, ctx->resident[0][mixed],
                                   ctx->forced_grid).total;
    if (need > (size_t)STOKES_NOALLOC_SCRATCH_BYTES)
        return fail(STOKES_EWORKSPACE, "stokes_sl_eval_noalloc: these sizes need " + std::to_string(need) +
                                           " bytes of scratch, more than the library's " +
                                           std::to_string((size_t)STOKES_NOALLOC_SCRATCH_BYTES) +
                                           "-byte array (use stokes_sl_eval with a workspace)");
    if (!ctx->scratch)
        return fail(STOKES_EDEVICE, std::string("stokes_sl_eval_noalloc: no device address for the scratch "
                                                "array: ") + hipGetErrorString(ctx->scratch_status));
    return direct_eval(ctx, STOKES_KERNEL_SL, n_src, src_xyz, density, weight, nullptr, n_trg, trg_xyz,
                       1.0 / (8.0 * kPi * mu), excl, opts, vel_out, ctx->scratch,
                       (size_t)STOKES_NOALLOC_SCRATCH_BYTES, stream, /*allow_sym=*/false);
}

int stokes_dl_eval(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                   const double* weight, const double* normal, int64_t n_trg,
                   const double* trg_xyz, const stokes_exclusion* excl, const stokes_opts* opts,
                   double* vel_out, void* workspace, size_t ws_bytes, void* stream) {
    return direct_eval(ctx, STOKES_KERNEL_DL, n_src, src_xyz, density, weight, normal, n_trg,
                       trg_xyz, 6.0 / (8.0 * kPi), excl, opts, vel_out, workspace, ws_bytes, stream);
}

int stokes_p2p_plan_create(stokes_ctx* ctx, int32_t n_leaves, int64_t n_src, int64_t n_trg,
                           const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs,
                           const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist,
                           stokes_p2p_plan** plan) {
    if (!plan) return fail(STOKES_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    if (n_leaves < 0) return fail(STOKES_EINVAL, "n_leaves must be >= 0");
    if (n_ulist < 0) return fail(STOKES_EINVAL, "n_ulist must be >= 0");
    if (!src_leaf_ofs || !trg_leaf_ofs || !ulist_ofs)
        return fail(STOKES_EINVAL, "leaf offset arrays (n_leaves + 1 entries, host) must be non-NULL");
    if (n_ulist > 0 && !ulist) return fail(STOKES_EINVAL, "ulist must be non-NULL when n_ulist > 0");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    std::string err;
    rc = stokes::p2p_plan_build(ctx->device, n_leaves, n_src, n_trg, src_leaf_ofs, trg_leaf_ofs,
                                ulist_ofs, ulist, n_ulist, plan, err);
    if (rc) return fail(rc, "stokes_p2p_plan_create: " + err);
    return STOKES_OK;
}

void stokes_p2p_plan_destroy(stokes_p2p_plan* plan) {
    if (!plan) return;
    DeviceGuard dg((int)stokes::p2p_plan_info(plan, 4));
    stokes::p2p_plan_free(plan);
}

int stokes_p2p_plan_pairs(const stokes_p2p_plan* plan, int64_t* pairs) {
    if (!plan || !pairs) return fail(STOKES_EINVAL, "plan and pairs must be non-NULL");
    *pairs = stokes::p2p_plan_info(plan, 3);
    return STOKES_OK;
}

int stokes_p2p_plan_eval(stokes_ctx* ctx, const stokes_p2p_plan* plan, int32_t kernel,
                         int64_t n_src, const double* src_xyz, const double* density,
                         const double* weight, const double* normal, int64_t n_trg,
                         const double* trg_xyz, double mu, const stokes_exclusion* excl,
                         const stokes_opts* opts, double* vel_out, void* workspace, size_t ws_bytes,
                         void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!plan) return fail(STOKES_EINVAL, "plan is NULL");
    if (kernel != STOKES_KERNEL_SL && kernel != STOKES_KERNEL_DL)
        return fail(STOKES_EINVAL, "kernel must be STOKES_KERNEL_SL or STOKES_KERNEL_DL");
    if (kernel == STOKES_KERNEL_SL && !(isfinite(mu) && mu > 0.0))
        return fail(STOKES_EINVAL, "mu must be finite and > 0");
    if (stokes::p2p_plan_info(plan, 4) != ctx->device)
        return fail(STOKES_EINVAL, "the plan was built on another device");
    if (n_src != stokes::p2p_plan_info(plan, 0) || n_trg != stokes::p2p_plan_info(plan, 1))
        return fail(STOKES_EINVAL, "n_src / n_trg differ from the plan's");
    int rc = check_points(kernel, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz);
    if (rc) return rc;
    if (!arr_ok(vel_out, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "vel_out must be non-NULL and 8-byte aligned");
    Parsed p;
    rc = parse_common(excl, opts, n_src, n_trg, p);
    if (rc) return rc;
    const size_t vb = (size_t)3 * n_trg * sizeof(double), sb = (size_t)3 * n_src * sizeof(double);
    rc = check_no_alias(vel_out, vb, "vel_out",
                        {{src_xyz, sb}, {density, sb}, {weight, (size_t)n_src * 8}, {normal, kernel ? sb : 0},
                         {trg_xyz, vb}, {workspace, ws_bytes}});
    if (rc) return rc;
    const int mixed = p.precision == STOKES_MIXED;
    const int32_t nl = (int32_t)stokes::p2p_plan_info(plan, 2);
    rc = check_workspace(workspace, ws_bytes, stokes::p2p_workspace_bytes(kernel, mixed, n_src, n_trg, nl));
    if (rc) return rc;
    int32_t* pair_class = nullptr;
    if ((rc = pair_class_for(ctx, mixed, n_src, n_trg, &pair_class))) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_trg == 0) return STOKES_OK;
    if (n_src == 0)
        return p.accumulate ? STOKES_OK
                            : launch_status(stokes::launch_fill_zero(vel_out, 3 * n_trg, st), "stokes_p2p_plan_eval");
    const double pref = kernel == STOKES_KERNEL_SL ? 1.0 / (8.0 * kPi * mu) : 6.0 / (8.0 * kPi);
    stokes::SumInputs in = make_inputs(kernel, p, n_src, src_xyz, density, weight, normal, n_trg,
                                       trg_xyz, pref);
    in.pair_class = pair_class;
    return launch_status(stokes::launch_p2p(in, plan, vel_out, p.accumulate, workspace, st,
                                            stokes::next_timer(ctx)),
                         "stokes_p2p_plan_eval");
}

int stokes_p2p_leaf_eval(stokes_ctx* ctx, int32_t kernel, int64_t n_src, const double* src_xyz,
                         const double* density, const double* weight, const double* normal, int64_t n_trg,
                         const double* trg_xyz, int32_t n_leaves, const int64_t* src_leaf_ofs,
                         const int64_t* trg_leaf_ofs, const int64_t* ulist_ofs, const int32_t* ulist,
                         int64_t n_ulist, double mu, const stokes_exclusion* excl, const stokes_opts* opts,
                         double* vel_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (kernel != STOKES_KERNEL_SL && kernel != STOKES_KERNEL_DL)
        return fail(STOKES_EINVAL, "kernel must be STOKES_KERNEL_SL or STOKES_KERNEL_DL");
    if (kernel == STOKES_KERNEL_SL && !(isfinite(mu) && mu > 0.0))
        return fail(STOKES_EINVAL, "mu must be finite and > 0");
    if (n_leaves < 0) return fail(STOKES_EINVAL, "n_leaves must be >= 0");
    if (n_ulist < 0 || n_ulist > INT32_MAX) return fail(STOKES_EINVAL, "n_ulist must be in [0, 2^31)");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    if (n_src > INT32_MAX) return fail(STOKES_EUNSUPPORTED, "n_src must be below 2^31 for leaf sums");
    rc = check_points(kernel, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz);
    if (rc) return rc;
    if (!arr_ok(vel_out, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "vel_out must be non-NULL and 8-byte aligned");
    if (!arr_ok(src_leaf_ofs, (int64_t)n_leaves + 1, 8) || !arr_ok(trg_leaf_ofs, (int64_t)n_leaves + 1, 8) ||
        !arr_ok(ulist_ofs, (int64_t)n_leaves + 1, 8))
        return fail(STOKES_EINVAL, "src_leaf_ofs, trg_leaf_ofs and ulist_ofs must be non-NULL and 8-byte aligned");
    if (!arr_ok(ulist, n_ulist, 4)) return fail(STOKES_EINVAL, "ulist must be non-NULL and 4-byte aligned");
    Parsed p;
    rc = parse_common(excl, opts, n_src, n_trg, p);
    if (rc) return rc;
    const size_t vb = (size_t)3 * n_trg * sizeof(double), sb = (size_t)3 * n_src * sizeof(double);
    const size_t ob = (size_t)(n_leaves + 1) * sizeof(int64_t);
    rc = check_no_alias(vel_out, vb, "vel_out",
                        {{src_xyz, sb}, {density, sb}, {weight, (size_t)n_src * 8}, {normal, kernel ? sb : 0},
                         {trg_xyz, vb}, {workspace, ws_bytes}, {src_leaf_ofs, ob}, {trg_leaf_ofs, ob},
                         {ulist_ofs, ob}, {ulist, (size_t)n_ulist * 4}});
    if (rc) return rc;
    const int mixed = p.precision == STOKES_MIXED;
    rc = check_workspace(workspace, ws_bytes, stokes::p2p_workspace_bytes(kernel, mixed, n_src, n_trg, n_leaves));
    if (rc) return rc;
    int32_t* pair_class = nullptr;
    if ((rc = pair_class_for(ctx, mixed, n_src, n_trg, &pair_class))) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_trg == 0) return STOKES_OK;
    if (n_src == 0)
        return p.accumulate ? STOKES_OK
                            : launch_status(stokes::launch_fill_zero(vel_out, 3 * n_trg, st), "stokes_p2p_leaf_eval");
    const double pref = kernel == STOKES_KERNEL_SL ? 1.0 / (8.0 * kPi * mu) : 6.0 / (8.0 * kPi);
    stokes::SumInputs in = make_inputs(kernel, p, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz, pref);
    in.pair_class = pair_class;
    return launch_status(stokes::launch_p2p_csr(in, n_leaves, src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, n_ulist,
                                                vel_out, p.accumulate, workspace, st, stokes::next_timer(ctx)),
                         "stokes_p2p_leaf_eval");
}

static int p2p_vjp_eval(stokes_ctx* ctx, int kernel, int64_t n_src, const double* src_xyz, const double* density,
                        const double* weight, const double* normal, int64_t n_trg, const double* trg_xyz,
                        int32_t n_leaves, const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs,
                        const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist, double pref,
                        const stokes_exclusion* excl, const stokes_opts* opts, const double* grad_vel,
                        double* grad_density, double* grad_src_xyz, double* grad_trg_xyz, void* workspace,
                        size_t ws_bytes, void* stream, const char* name) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (n_leaves < 0) return fail(STOKES_EINVAL, "n_leaves must be >= 0");
    if (n_ulist < 0 || n_ulist > INT32_MAX) return fail(STOKES_EINVAL, "n_ulist must be in [0, 2^31)");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    rc = check_points(kernel, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz);
    if (rc) return rc;
    if (!arr_ok(grad_vel, 3 * n_trg, 8) || (n_trg > 0 && !grad_vel))
        return fail(STOKES_EINVAL, "grad_vel must be non-NULL and 8-byte aligned");
    if (!arr_ok(src_leaf_ofs, (int64_t)n_leaves + 1, 8) || !arr_ok(trg_leaf_ofs, (int64_t)n_leaves + 1, 8) ||
        !arr_ok(ulist_ofs, (int64_t)n_leaves + 1, 8))
        return fail(STOKES_EINVAL, "src_leaf_ofs, trg_leaf_ofs and ulist_ofs must be non-NULL and 8-byte aligned");
    if (!arr_ok(ulist, n_ulist, 4)) return fail(STOKES_EINVAL, "ulist must be non-NULL and 4-byte aligned");
    for (const double* g : {(const double*)grad_density, (const double*)grad_src_xyz, (const double*)grad_trg_xyz})
        if (g && !aligned(g, 8)) return fail(STOKES_EINVAL, "gradient outputs must be 8-byte aligned");
    Parsed p;
    if ((rc = parse_common(excl, opts, n_src, n_trg, p))) return rc;
    const size_t sb = (size_t)3 * n_src * 8, tb = (size_t)3 * n_trg * 8, ob = (size_t)(n_leaves + 1) * 8;
    struct Out { void* ptr; size_t bytes; const char* name; };
    const Out outs[3] = {{grad_density, sb, "grad_density"}, {grad_src_xyz, sb, "grad_src_xyz"},
                         {grad_trg_xyz, tb, "grad_trg_xyz"}};
    for (int a = 0; a < 3; ++a) {
        if (!outs[a].ptr) continue;
        if ((rc = check_no_alias(outs[a].ptr, outs[a].bytes, outs[a].name,
                                 {{src_xyz, sb}, {density, sb}, {weight, (size_t)n_src * 8}, {normal, sb}, {trg_xyz, tb},
                                  {grad_vel, tb}, {workspace, ws_bytes}, {src_leaf_ofs, ob}, {trg_leaf_ofs, ob},
                                  {ulist_ofs, ob}, {ulist, (size_t)n_ulist * 4}})))
            return rc;
        for (int b = a + 1; b < 3; ++b)
            if (outs[b].ptr && overlaps(outs[a].ptr, outs[a].bytes, outs[b].ptr, outs[b].bytes))
                return fail(STOKES_EINVAL, std::string(outs[a].name) + " overlaps " + outs[b].name);
    }
    rc = check_workspace(workspace, ws_bytes, stokes::p2p_vjp_workspace_bytes(kernel, n_src, n_trg, n_leaves, n_ulist));
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_src == 0 || n_trg == 0) {            // zero gradients (kept when accumulating)
        if (p.accumulate) return STOKES_OK;
        hipError_t e = hipSuccess;
        if (grad_density && e == hipSuccess) e = stokes::launch_fill_zero(grad_density, 3 * n_src, st);
        if (grad_src_xyz && e == hipSuccess) e = stokes::launch_fill_zero(grad_src_xyz, 3 * n_src, st);
        if (grad_trg_xyz && e == hipSuccess) e = stokes::launch_fill_zero(grad_trg_xyz, 3 * n_trg, st);
        return launch_status(e, name);
    }
    Parsed pf = p;
    pf.precision = STOKES_FP64;                // adjoints run in float64
    stokes::SumInputs in = make_inputs(kernel, pf, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz, pref);
    return launch_status(stokes::launch_p2p_vjp(in, n_leaves, src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, n_ulist,
                                                grad_vel, grad_density, grad_src_xyz, grad_trg_xyz, p.accumulate,
                                                workspace, st),
                         name);
}

int stokes_p2p_sl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                      const double* weight, int64_t n_trg, const double* trg_xyz, int32_t n_leaves,
                      const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs, const int64_t* ulist_ofs,
                      const int32_t* ulist, int64_t n_ulist, double mu, const stokes_exclusion* excl,
                      const stokes_opts* opts, const double* grad_vel, double* grad_density, double* grad_src_xyz,
                      double* grad_trg_xyz, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!(isfinite(mu) && mu > 0.0)) return fail(STOKES_EINVAL, "mu must be finite and > 0");
    return p2p_vjp_eval(ctx, STOKES_KERNEL_SL, n_src, src_xyz, density, weight, nullptr, n_trg, trg_xyz, n_leaves,
                        src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, n_ulist, 1.0 / (8.0 * kPi * mu), excl, opts,
                        grad_vel, grad_density, grad_src_xyz, grad_trg_xyz, workspace, ws_bytes, stream,
                        "stokes_p2p_sl_vjp");
}

int stokes_p2p_dl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                      const double* weight, const double* normal, int64_t n_trg, const double* trg_xyz,
                      int32_t n_leaves, const int64_t* src_leaf_ofs, const int64_t* trg_leaf_ofs,
                      const int64_t* ulist_ofs, const int32_t* ulist, int64_t n_ulist, const stokes_exclusion* excl,
                      const stokes_opts* opts, const double* grad_vel, double* grad_density, double* grad_src_xyz,
                      double* grad_trg_xyz, void* workspace, size_t ws_bytes, void* stream) {
    return p2p_vjp_eval(ctx, STOKES_KERNEL_DL, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz, n_leaves,
                        src_leaf_ofs, trg_leaf_ofs, ulist_ofs, ulist, n_ulist, 6.0 / (8.0 * kPi), excl, opts,
                        grad_vel, grad_density, grad_src_xyz, grad_trg_xyz, workspace, ws_bytes, stream,
                        "stokes_p2p_dl_vjp");
}

static int vjp_eval(stokes_ctx* ctx, int kernel, int64_t n_src, const double* src_xyz,
                    const double* density, const double* weight, const double* normal, int64_t n_trg,
                    const double* trg_xyz, double pref, const stokes_exclusion* excl,
                    const stokes_opts* opts, const double* grad_vel, double* grad_density,
                    double* grad_src_xyz, double* grad_trg_xyz, void* workspace, size_t ws_bytes,
                    void* stream) {
    const char* name = kernel ? "stokes_dl_vjp" : "stokes_sl_vjp";
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    rc = check_points(kernel, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz);
    if (rc) return rc;
    if (!arr_ok(grad_vel, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "grad_vel must be non-NULL and 8-byte aligned");
    for (const double* g : {grad_density, grad_src_xyz, grad_trg_xyz})
        if (g && !aligned(g, 8)) return fail(STOKES_EINVAL, "gradient outputs must be 8-byte aligned");
    Parsed p;
    rc = parse_common(excl, opts, n_src, n_trg, p);
    if (rc) return rc;
    const size_t sb = (size_t)3 * n_src * 8, tb = (size_t)3 * n_trg * 8;
    const bool shared = src_xyz == trg_xyz && n_src == n_trg &&
                        (p.excl == STOKES_EXCL_NONE || p.src_group == p.trg_group);
    const bool combined = grad_src_xyz && grad_src_xyz == grad_trg_xyz;
    if (combined && !shared)
        return fail(STOKES_EINVAL, "grad_src_xyz and grad_trg_xyz may be one array only when sources and "
                                   "targets are the same point set (and group array)");
    const std::initializer_list<std::pair<const void*, size_t>> inputs = {
        {src_xyz, sb}, {density, sb}, {weight, (size_t)n_src * 8}, {normal, kernel ? sb : 0},
        {trg_xyz, tb}, {grad_vel, tb}, {workspace, ws_bytes}};
    if ((rc = check_no_alias(grad_density, sb, "grad_density", inputs))) return rc;
    if ((rc = check_no_alias(grad_src_xyz, sb, "grad_src_xyz", inputs))) return rc;
    if ((rc = check_no_alias(grad_trg_xyz, tb, "grad_trg_xyz", inputs))) return rc;
    if (overlaps(grad_density, sb, grad_src_xyz, sb) ||
        overlaps(grad_density, sb, grad_trg_xyz, tb) ||
        (!combined && overlaps(grad_src_xyz, sb, grad_trg_xyz, tb)))
        return fail(STOKES_EINVAL, "gradient outputs overlap each other");
    const size_t need = stokes::vjp_workspace_bytes(kernel, n_src, n_trg, ctx->vjp_resident);
    rc = check_workspace(workspace, ws_bytes, need);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_src == 0 || n_trg == 0) {           // empty sums: zero (or keep, when accumulating)
        if (p.accumulate) return STOKES_OK;
        hipError_t e = hipSuccess;
        if (grad_density) e = stokes::launch_fill_zero(grad_density, 3 * n_src, st);
        if (e == hipSuccess && grad_src_xyz) e = stokes::launch_fill_zero(grad_src_xyz, 3 * n_src, st);
        if (e == hipSuccess && grad_trg_xyz && !combined)
            e = stokes::launch_fill_zero(grad_trg_xyz, 3 * n_trg, st);
        return launch_status(e, name);
    }
    stokes::VjpInputs in{};
    in.n_src = n_src;
    in.n_trg = n_trg;
    in.src_xyz = src_xyz;
    in.density = density;
    in.weight = weight;
    in.normal = normal;
    in.trg_xyz = trg_xyz;
    in.grad_vel = grad_vel;
    in.excl = p.excl;
    in.src_group = p.src_group;
    in.trg_group = p.trg_group;
    in.pref = pref;
    in.accumulate = p.accumulate;
    in.grad_density = grad_density;
    in.grad_src = grad_src_xyz;
    in.grad_trg = grad_trg_xyz;
    const stokes::KernelTimer timer = stokes::next_timer(ctx);
    // a shared point set with one combined position gradient takes the
    // each-pair-once adjoint when the workspace has room for it
    if (kernel == STOKES_KERNEL_SL && shared && combined &&
        sym_available(ctx, STOKES_KERNEL_SL, 0, n_src, n_trg)) {
        const stokes::SymPlan sp = stokes::plan_sym(1, n_src, ctx->sym_resident[1], ctx->forced_grid);
        if (ws_bytes >= sp.total) {
            const stokes::SumInputs si = make_inputs(STOKES_KERNEL_SL, p, n_src, src_xyz, density, weight,
                                                     nullptr, n_trg, trg_xyz, pref);
            if (timer.on()) (void)hipEventRecord(timer.start, st);
            hipError_t e = stokes::launch_sym_vjp(si, sp, grad_vel, grad_density, grad_src_xyz, p.accumulate,
                                                  workspace, st, stokes::KernelTimer{});
            if (timer.on()) (void)hipEventRecord(timer.stop, st);
            return launch_status(e, name);
        }
    }
    if (timer.on()) (void)hipEventRecord(timer.start, st);
    hipError_t e = kernel ? stokes::launch_dl_vjp(in, ctx->vjp_resident, combined, workspace, st)
                          : stokes::launch_sl_vjp(in, ctx->vjp_resident, combined, workspace, st);
    if (timer.on()) (void)hipEventRecord(timer.stop, st);
    return launch_status(e, name);
}

int stokes_sl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                  const double* weight, int64_t n_trg, const double* trg_xyz, double mu,
                  const stokes_exclusion* excl, const stokes_opts* opts, const double* grad_vel,
                  double* grad_density, double* grad_src_xyz, double* grad_trg_xyz, void* workspace,
                  size_t ws_bytes, void* stream) {
    if (!(isfinite(mu) && mu > 0.0)) return fail(STOKES_EINVAL, "mu must be finite and > 0");
    return vjp_eval(ctx, STOKES_KERNEL_SL, n_src, src_xyz, density, weight, nullptr, n_trg, trg_xyz,
                    1.0 / (8.0 * kPi * mu), excl, opts, grad_vel, grad_density, grad_src_xyz,
                    grad_trg_xyz, workspace, ws_bytes, stream);
}

int stokes_dl_vjp(stokes_ctx* ctx, int64_t n_src, const double* src_xyz, const double* density,
                  const double* weight, const double* normal, int64_t n_trg,
                  const double* trg_xyz, const stokes_exclusion* excl, const stokes_opts* opts,
                  const double* grad_vel, double* grad_density, double* grad_src_xyz,
                  double* grad_trg_xyz, void* workspace, size_t ws_bytes, void* stream) {
    return vjp_eval(ctx, STOKES_KERNEL_DL, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz,
                    6.0 / (8.0 * kPi), excl, opts, grad_vel, grad_density, grad_src_xyz, grad_trg_xyz,
                    workspace, ws_bytes, stream);
}

int stokes_patch_upsample(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                          const double* node_xyz, const double* density, double* fine_xyz,
                          double* fine_density, double* fine_weight, double* fine_normal,
                          double* patch_size, void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    stokes::PatchRule R;
    int rc = parse_patch_rule(rule, false, R);
    if (rc) return rc;
    CheckpointLayout lay;
    if ((rc = checkpoint_layout(ctx, n_patches, R, 0, 0, false, lay))) return rc;
    const int64_t nn = lay.n_nodes, nf = lay.n_fine;
    if (!arr_ok(node_xyz, 3 * nn, 8)) return fail(STOKES_EINVAL, "node_xyz must be non-NULL and 8-byte aligned");
    if (density && !aligned(density, 8)) return fail(STOKES_EINVAL, "density must be 8-byte aligned");
    if (!arr_ok(fine_xyz, 3 * nf, 8) || !arr_ok(fine_weight, nf, 8) || !arr_ok(fine_normal, 3 * nf, 8) ||
        !arr_ok(patch_size, n_patches, 8))
        return fail(STOKES_EINVAL, "fine_xyz, fine_weight, fine_normal and patch_size must be non-NULL and "
                                   "8-byte aligned");
    if (density && !arr_ok(fine_density, 3 * nf, 8))
        return fail(STOKES_EINVAL, "fine_density must be non-NULL and 8-byte aligned when density is given");
    const size_t nb = (size_t)3 * nn * 8, fb = (size_t)3 * nf * 8;
    const std::pair<const void*, size_t> outs[] = {{fine_xyz, fb},
                                                   {density ? fine_density : nullptr, fb},
                                                   {fine_weight, (size_t)nf * 8},
                                                   {fine_normal, fb},
                                                   {patch_size, (size_t)n_patches * 8}};
    for (int i = 0; i < 5; ++i) {
        if ((rc = check_no_alias(outs[i].first, outs[i].second, "an upsampling output",
                                 {{node_xyz, nb}, {density, density ? nb : 0}})))
            return rc;
        for (int j = 0; j < i; ++j)
            if (overlaps(outs[i].first, outs[i].second, outs[j].first, outs[j].second))
                return fail(STOKES_EINVAL, "upsampling outputs overlap each other");
    }
    if (n_patches == 0) return STOKES_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    return launch_status(stokes::launch_upsample(R, n_patches, node_xyz, density, fine_xyz,
                                                 density ? fine_density : nullptr, fine_weight, fine_normal,
                                                 patch_size, static_cast<hipStream_t>(stream)),
                         "stokes_patch_upsample");
}

int stokes_checkpoint_workspace_size(const stokes_ctx* ctx, int64_t n_patches,
                                     const stokes_patch_rule* rule, int64_t n_trg,
                                     const stokes_opts* opts, size_t* bytes) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!bytes) return fail(STOKES_EINVAL, "bytes is NULL");
    stokes::PatchRule R;
    int rc = parse_patch_rule(rule, true, R);
    if (rc) return rc;
    Parsed p;
    if ((rc = parse_common(nullptr, opts, 0, 0, p))) return rc;
    CheckpointLayout lay;
    if ((rc = checkpoint_layout(ctx, n_patches, R, n_trg, p.precision == STOKES_MIXED, true, lay))) return rc;
    *bytes = lay.total;
    return STOKES_OK;
}

int stokes_dl_checkpoint_eval(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                              const double* node_xyz, const double* density, int64_t n_trg,
                              const int32_t* trg_patch, const double* trg_uvd,
                              const stokes_opts* opts, double* vel_out, double* check_xyz_out,
                              double* check_vel_out, void* workspace, size_t ws_bytes,
                              void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    stokes::PatchRule R;
    int rc = parse_patch_rule(rule, true, R);
    if (rc) return rc;
    Parsed p;
    if ((rc = parse_common(nullptr, opts, 0, 0, p))) return rc;
    CheckpointLayout lay;
    if ((rc = checkpoint_layout(ctx, n_patches, R, n_trg, p.precision == STOKES_MIXED, true, lay))) return rc;
    if (n_patches == 0 && n_trg > 0) return fail(STOKES_EINVAL, "targets need at least one patch (n_patches == 0)");
    if ((trg_patch == nullptr) != (trg_uvd == nullptr))
        return fail(STOKES_EINVAL, "trg_patch and trg_uvd must both be given or both be NULL");
    if (!trg_patch && n_trg != lay.n_nodes)
        return fail(STOKES_EINVAL, "without trg_patch the targets are the n_patches*q*q nodes: n_trg must equal "
                                   "that count");
    const int64_t nn = lay.n_nodes;
    if (!arr_ok(node_xyz, 3 * nn, 8)) return fail(STOKES_EINVAL, "node_xyz must be non-NULL and 8-byte aligned");
    if (!arr_ok(density, 3 * nn, 8)) return fail(STOKES_EINVAL, "density must be non-NULL and 8-byte aligned");
    if (trg_patch && (!arr_ok(trg_patch, n_trg, 4) || !arr_ok(trg_uvd, 3 * n_trg, 8)))
        return fail(STOKES_EINVAL, "trg_patch must be 4-byte and trg_uvd 8-byte aligned");
    if (!arr_ok(vel_out, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "vel_out must be non-NULL and 8-byte aligned");
    if ((check_xyz_out && !aligned(check_xyz_out, 8)) || (check_vel_out && !aligned(check_vel_out, 8)))
        return fail(STOKES_EINVAL, "check_xyz_out and check_vel_out must be 8-byte aligned");
    const size_t nb = (size_t)3 * nn * 8, tb = (size_t)3 * n_trg * 8, cb = (size_t)3 * lay.n_check * 8;
    const std::initializer_list<std::pair<const void*, size_t>> inputs = {
        {node_xyz, nb}, {density, nb}, {trg_patch, trg_patch ? (size_t)n_trg * 4 : 0},
        {trg_uvd, trg_uvd ? tb : 0}, {workspace, ws_bytes}};
    if ((rc = check_no_alias(vel_out, tb, "vel_out", inputs))) return rc;
    if ((rc = check_no_alias(check_xyz_out, cb, "check_xyz_out", inputs))) return rc;
    if ((rc = check_no_alias(check_vel_out, cb, "check_vel_out", inputs))) return rc;
    if (overlaps(vel_out, tb, check_xyz_out, cb) || overlaps(vel_out, tb, check_vel_out, cb) ||
        overlaps(check_xyz_out, cb, check_vel_out, cb))
        return fail(STOKES_EINVAL, "outputs overlap each other");
    if ((rc = check_workspace(workspace, ws_bytes, lay.total))) return rc;
    if (n_trg == 0) return STOKES_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    return launch_status(checkpoint_run(ctx, R, lay, n_patches, node_xyz, density, n_trg, trg_patch, trg_uvd, p,
                                        vel_out, check_xyz_out, check_vel_out, static_cast<char*>(workspace),
                                        static_cast<hipStream_t>(stream)),
                         "stokes_dl_checkpoint_eval");
}

int stokes_bie_workspace_size(const stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule,
                              int32_t max_iter, const stokes_opts* opts, size_t* bytes) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!bytes) return fail(STOKES_EINVAL, "bytes is NULL");
    stokes::PatchRule R;
    int rc = parse_patch_rule(rule, true, R);
    if (rc) return rc;
    Parsed p;
    if ((rc = parse_common(nullptr, opts, 0, 0, p))) return rc;
    BieLayout lay;
    if ((rc = bie_layout(ctx, n_patches, R, max_iter, p.precision == STOKES_MIXED, lay))) return rc;
    *bytes = lay.total;
    return STOKES_OK;
}

// Shared checks of the operator and the solve: rule, options, layout, node
// array, one input and one output vector of 3 * nodes doubles, workspace.
static int bie_prepare(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule, int32_t max_iter,
                       const double* node_xyz, const double* in, const char* in_name, const stokes_opts* opts,
                       const double* out, const char* out_name, void* workspace, size_t ws_bytes,
                       stokes::PatchRule& R, Parsed& p, BieLayout& lay) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    int rc = parse_patch_rule(rule, true, R);
    if (rc) return rc;
    if ((rc = parse_common(nullptr, opts, 0, 0, p))) return rc;
    if ((rc = bie_layout(ctx, n_patches, R, max_iter, p.precision == STOKES_MIXED, lay))) return rc;
    const int64_t n3 = lay.n3;
    if (!arr_ok(node_xyz, n3, 8)) return fail(STOKES_EINVAL, "node_xyz must be non-NULL and 8-byte aligned");
    if (!arr_ok(in, n3, 8)) return fail(STOKES_EINVAL, std::string(in_name) + " must be non-NULL and 8-byte aligned");
    if (!arr_ok(out, n3, 8))
        return fail(STOKES_EINVAL, std::string(out_name) + " must be non-NULL and 8-byte aligned");
    const size_t vb = (size_t)n3 * 8;
    if ((rc = check_no_alias(out, vb, out_name, {{node_xyz, vb}, {in, vb}, {workspace, ws_bytes}}))) return rc;
    return check_workspace(workspace, ws_bytes, lay.total);
}

int stokes_bie_apply(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule, const double* node_xyz,
                     const double* phi, const stokes_opts* opts, double* out, void* workspace, size_t ws_bytes,
                     void* stream) {
    stokes::PatchRule R;
    Parsed p;
    BieLayout lay;
    int rc = bie_prepare(ctx, n_patches, rule, 0, node_xyz, phi, "phi", opts, out, "out", workspace, ws_bytes, R, p,
                         lay);
    if (rc) return rc;
    if (lay.n3 == 0) return STOKES_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    hipError_t e = bie_geometry(R, lay, n_patches, node_xyz, ws, st);
    if (e == hipSuccess) e = bie_apply_run(ctx, R, lay, n_patches, node_xyz, phi, p, out, ws, 0, st);
    return launch_status(e, "stokes_bie_apply");
}

int stokes_bie_solve(stokes_ctx* ctx, int64_t n_patches, const stokes_patch_rule* rule, const double* node_xyz,
                     const double* g, int32_t max_iter, double rtol, const stokes_opts* opts, double* phi_out,
                     int32_t* iterations, double* residual_history, void* workspace, size_t ws_bytes,
                     void* stream) {
    if (max_iter < 1) return fail(STOKES_EINVAL, "max_iter must be in [1, " + std::to_string(stokes::kMaxKrylov) + "]");
    if (!(rtol >= 0.0) || !isfinite(rtol)) return fail(STOKES_EINVAL, "rtol must be finite and >= 0");
    if (!iterations) return fail(STOKES_EINVAL, "iterations is NULL");
    if (opts && opts->accumulate) return fail(STOKES_EINVAL, "opts.accumulate must be 0 for the solve");
    stokes::PatchRule R;
    Parsed p;
    BieLayout lay;
    int rc = bie_prepare(ctx, n_patches, rule, max_iter, node_xyz, g, "g", opts, phi_out, "phi_out", workspace,
                         ws_bytes, R, p, lay);
    if (rc) return rc;
    *iterations = 0;
    if (residual_history) residual_history[0] = 1.0;
    if (lay.n3 == 0) return STOKES_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    const int64_t n3 = lay.n3;
    double* V = reinterpret_cast<double*>(ws + lay.off_V);
    double* w = reinterpret_cast<double*>(ws + lay.off_w);
    double* part = reinterpret_cast<double*>(ws + lay.off_part);
    double* dots = reinterpret_cast<double*>(ws + lay.off_dots);
    double* coef = reinterpret_cast<double*>(ws + lay.off_coef);
    auto status = [](hipError_t e) { return launch_status(e, "stokes_bie_solve"); };
    auto read = [&](double* host, int count) -> hipError_t {
        hipError_t e = hipMemcpyAsync(host, dots, (size_t)count * 8, hipMemcpyDeviceToHost, st);
        return e == hipSuccess ? hipStreamSynchronize(st) : e;
    };

    // beta = |g|, v_0 = g / beta
    hipError_t e = bie_geometry(R, lay, n_patches, node_xyz, ws, st);
    if (e == hipSuccess) e = stokes::launch_multi_dot(g, n3, 1, g, n3, part, dots, st);
    double beta2 = 0.0;
    if (e == hipSuccess) e = read(&beta2, 1);
    if (e != hipSuccess) return status(e);
    if (!isfinite(beta2)) return fail(STOKES_EINVAL, "g holds non-finite values");
    const double beta = sqrt(beta2);
    if (beta == 0.0) return status(stokes::launch_fill_zero(phi_out, n3, st));
    if ((e = stokes::launch_scale(V, g, 1.0 / beta, n3, st)) != hipSuccess) return status(e);

    // Arnoldi with classical Gram-Schmidt applied twice; Givens rotations on
    // the Hessenberg matrix on the host.
    const int m = max_iter;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), sv(m + 1, 0.0), hd(2 * m + 2);
    auto h = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    sv[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
        const double* vj = V + (int64_t)j * n3;
        const int nv = j + 1;
        e = bie_apply_run(ctx, R, lay, n_patches, node_xyz, vj, p, w, ws, 2 * m + 2, st);
        for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            e = stokes::launch_multi_dot(V, n3, nv, w, n3, part, dots + pass * nv, st);
            if (e == hipSuccess) e = stokes::launch_combo_sub(w, V, n3, nv, dots + pass * nv, n3, st);
        }
        if (e == hipSuccess) e = stokes::launch_multi_dot(w, n3, 1, w, n3, part, dots + 2 * nv, st);
        if (e == hipSuccess) e = read(hd.data(), 2 * nv + 1);
        if (e != hipSuccess) return status(e);
        for (int i = 0; i < nv; ++i) h(i, j) = hd[i] + hd[nv + i];
        const double hnext = sqrt(fmax(hd[2 * nv], 0.0));
        h(j + 1, j) = hnext;
        if (!isfinite(hnext)) return fail(STOKES_EDEVICE, "stokes_bie_solve: non-finite Krylov vector");
        for (int i = 0; i < j; ++i) {
            const double a = h(i, j), b = h(i + 1, j);
            h(i, j) = cs[i] * a + sn[i] * b;
            h(i + 1, j) = -sn[i] * a + cs[i] * b;
        }
        const double den = hypot(h(j, j), h(j + 1, j));
        cs[j] = den > 0.0 ? h(j, j) / den : 1.0;
        sn[j] = den > 0.0 ? h(j + 1, j) / den : 0.0;
        h(j, j) = den;
        h(j + 1, j) = 0.0;
        sv[j + 1] = -sn[j] * sv[j];
        sv[j] = cs[j] * sv[j];
        k = j + 1;
        const double res = fabs(sv[j + 1]) / beta;
        if (residual_history) residual_history[k] = res;
        if (res <= rtol || hnext == 0.0 || k == m) break;
        if ((e = stokes::launch_scale(V + (int64_t)k * n3, w, 1.0 / hnext, n3, st)) != hipSuccess) return status(e);
    }
    // y = H_k^{-1} s by back substitution, phi = V_k y
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
        double acc = sv[i];
        for (int l = i + 1; l < k; ++l) acc -= h(i, l) * y[l];
        y[i] = h(i, i) != 0.0 ? acc / h(i, i) : 0.0;
    }
    e = hipMemcpyAsync(coef, y.data(), (size_t)k * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = stokes::launch_combo_set(phi_out, V, n3, k, coef, n3, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *iterations = k;
    return status(e);
}

int stokes_space_time_boxes(stokes_ctx* ctx, int32_t n_meshes, const int64_t* mesh_ofs, int64_t n_points,
                            const double* x0, const double* x1, double inflate, double* box_lo, double* box_hi,
                            void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (n_meshes < 0) return fail(STOKES_EINVAL, "n_meshes must be >= 0");
    int rc = check_sizes(n_points, 0);
    if (rc) return rc;
    if (!isfinite(inflate) || inflate < 0.0) return fail(STOKES_EINVAL, "inflate must be finite and >= 0");
    if (n_meshes > 0 && (!mesh_ofs || !aligned(mesh_ofs, 8)))
        return fail(STOKES_EINVAL, "mesh_ofs must be non-NULL and 8-byte aligned");
    if (!arr_ok(x0, 3 * n_points, 8)) return fail(STOKES_EINVAL, "x0 must be non-NULL and 8-byte aligned");
    if (x1 && !aligned(x1, 8)) return fail(STOKES_EINVAL, "x1 must be 8-byte aligned");
    if (!arr_ok(box_lo, 3 * (int64_t)n_meshes, 8) || !arr_ok(box_hi, 3 * (int64_t)n_meshes, 8))
        return fail(STOKES_EINVAL, "box_lo and box_hi must be non-NULL and 8-byte aligned");
    const size_t pb = (size_t)3 * n_points * 8, bb = (size_t)3 * n_meshes * 8;
    const std::initializer_list<std::pair<const void*, size_t>> inputs = {
        {mesh_ofs, (size_t)(n_meshes + 1) * 8}, {x0, pb}, {x1, x1 ? pb : 0}};
    if ((rc = check_no_alias(box_lo, bb, "box_lo", inputs))) return rc;
    if ((rc = check_no_alias(box_hi, bb, "box_hi", inputs))) return rc;
    if (overlaps(box_lo, bb, box_hi, bb)) return fail(STOKES_EINVAL, "box_lo and box_hi overlap");
    if (n_meshes == 0) return STOKES_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    return launch_status(stokes::launch_space_time_boxes(n_meshes, mesh_ofs, n_points, x0, x1, inflate, box_lo,
                                                         box_hi, static_cast<hipStream_t>(stream)),
                         "stokes_space_time_boxes");
}

int stokes_collision_workspace_size(const stokes_ctx* ctx, int32_t n_boxes, int64_t max_entries, size_t* bytes) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!bytes) return fail(STOKES_EINVAL, "bytes is NULL");
    if (n_boxes < 0) return fail(STOKES_EINVAL, "n_boxes must be >= 0");
    if (max_entries < 0 || max_entries > ((int64_t)1 << 31))
        return fail(STOKES_EINVAL, "max_entries must be in [0, 2^31]");
    *bytes = stokes::candidate_layout(n_boxes, max_entries).total;
    return STOKES_OK;
}

int stokes_collision_candidates(stokes_ctx* ctx, int32_t n_boxes, const double* box_lo, const double* box_hi,
                                double cell_size, int64_t max_entries, int32_t* pairs_out, int64_t capacity,
                                int64_t* n_pairs, int64_t* n_entries, void* workspace, size_t ws_bytes,
                                void* stream) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (n_boxes < 0) return fail(STOKES_EINVAL, "n_boxes must be >= 0");
    if (!(isfinite(cell_size) && cell_size > 0.0)) return fail(STOKES_EINVAL, "cell_size must be finite and > 0");
    if (max_entries < 0 || max_entries > ((int64_t)1 << 31))
        return fail(STOKES_EINVAL, "max_entries must be in [0, 2^31]");
    if (capacity < 0) return fail(STOKES_EINVAL, "capacity must be >= 0");
    if (!n_pairs) return fail(STOKES_EINVAL, "n_pairs is NULL");
    if (!arr_ok(box_lo, 3 * (int64_t)n_boxes, 8) || !arr_ok(box_hi, 3 * (int64_t)n_boxes, 8))
        return fail(STOKES_EINVAL, "box_lo and box_hi must be non-NULL and 8-byte aligned");
    if (!arr_ok(pairs_out, 2 * capacity, 4))
        return fail(STOKES_EINVAL, "pairs_out must be non-NULL and 4-byte aligned when capacity > 0");
    const size_t bb = (size_t)3 * n_boxes * 8;
    int rc = check_no_alias(pairs_out, (size_t)2 * capacity * 4, "pairs_out",
                            {{box_lo, bb}, {box_hi, bb}, {workspace, ws_bytes}});
    if (rc) return rc;
    const stokes::CandidateLayout lay = stokes::candidate_layout(n_boxes, max_entries);
    if ((rc = check_workspace(workspace, ws_bytes, lay.total))) return rc;
    *n_pairs = 0;
    if (n_entries) *n_entries = 0;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    stokes::CandidateMeta meta{};
    hipError_t e = stokes::candidate_phase1(n_boxes, box_lo, box_hi, cell_size, ws, lay, &meta, st);
    if (e != hipSuccess) return launch_status(e, "stokes_collision_candidates");
    if (n_entries) *n_entries = meta.entries;
    if (meta.overflow)
        return fail(STOKES_EUNSUPPORTED, "a box corner is not finite or lies 2^21 or more cells from the origin "
                                         "(cell_size too small)");
    if (meta.entries > max_entries)
        return fail(STOKES_EWORKSPACE, "max_entries " + std::to_string(max_entries) + " < the " +
                                           std::to_string(meta.entries) + " (box, cell) entries needed");
    int64_t np = 0;
    e = stokes::candidate_phase2(n_boxes, meta, ws, lay, &np, st);
    if (e == hipSuccess) e = stokes::candidate_phase3(n_boxes, meta, ws, lay, pairs_out, capacity, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *n_pairs = np;
    return launch_status(e, "stokes_collision_candidates");
}

int stokes_fmm_plan_create(stokes_ctx* ctx, int32_t order, stokes_fmm_plan** plan) {
    if (!plan) return fail(STOKES_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (order < stokes::kFmmMinOrder || order > stokes::kFmmMaxOrder)
        return fail(STOKES_EINVAL, "order must be in [" + std::to_string(stokes::kFmmMinOrder) + ", " +
                                       std::to_string(stokes::kFmmMaxOrder) + "]");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    std::string err;
    int rc;
    try {
        rc = stokes::fmm_plan_build(ctx->device, order, plan, err);
    } catch (const std::exception& ex) {           // host allocation of the operators
        rc = -1;
        err = ex.what();
    }
    if (rc != 0) return fail(STOKES_EDEVICE, "stokes_fmm_plan_create: " + err);
    return STOKES_OK;
}

void stokes_fmm_plan_destroy(stokes_fmm_plan* plan) {
    if (!plan) return;
    DeviceGuard dg(stokes::fmm_plan_device(plan));
    stokes::fmm_plan_free(plan);
}

static int fmm_check_sizes(const stokes_fmm_plan* plan, int64_t n_src, int64_t n_trg, int32_t depth) {
    if (!plan) return fail(STOKES_EINVAL, "plan is NULL");
    int rc = check_sizes(n_src, n_trg);
    if (rc) return rc;
    if (depth < stokes::kFmmMinDepth || depth > stokes::kFmmMaxDepth)
        return fail(STOKES_EINVAL, "depth must be in [" + std::to_string(stokes::kFmmMinDepth) + ", " +
                                       std::to_string(stokes::kFmmMaxDepth) + "]");
    return STOKES_OK;
}

// Groups of the FMM's same-group rule (0: no rule); the rule needs n_groups > 0.
static int fmm_groups(const stokes_exclusion* excl, int32_t* n_groups) {
    *n_groups = 0;
    if (!excl || excl->mode == STOKES_EXCL_NONE) return STOKES_OK;
    if (excl->mode != STOKES_EXCL_SAME_GROUP)
        return fail(STOKES_EINVAL, "exclusion.mode must be STOKES_EXCL_NONE or STOKES_EXCL_SAME_GROUP");
    if (excl->n_groups <= 0)
        return fail(STOKES_EINVAL, "the FMM's same-group rule needs n_groups > 0 (group ids in [0, n_groups))");
    *n_groups = excl->n_groups;
    return STOKES_OK;
}

// Workspace of an FMM evaluation: the FMM's, then the same-group correction's.
static size_t fmm_total_bytes(const stokes_fmm_plan* plan, int kernel, int64_t n_src, int64_t n_trg, int32_t depth,
                              int32_t n_groups, size_t* off_groups) {
    const size_t f = stokes::align_up(stokes::fmm_workspace_bytes(stokes::fmm_plan_order(plan), n_src, n_trg, depth), 256);
    if (off_groups) *off_groups = f;
    return f + stokes::same_group_workspace_bytes(kernel, n_src, n_trg, n_groups);
}

int stokes_fmm_workspace_size(const stokes_ctx* ctx, const stokes_fmm_plan* plan, int64_t n_src, int64_t n_trg,
                              int32_t depth, const stokes_exclusion* excl, size_t* bytes) {
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    if (!bytes) return fail(STOKES_EINVAL, "bytes is NULL");
    int rc = fmm_check_sizes(plan, n_src, n_trg, depth);
    if (rc) return rc;
    int32_t ng = 0;
    if ((rc = fmm_groups(excl, &ng))) return rc;
    // sized for the double layer, whose correction also gathers the normals
    *bytes = fmm_total_bytes(plan, STOKES_KERNEL_DL, n_src, n_trg, depth, ng, nullptr);
    return STOKES_OK;
}

static int fmm_eval(stokes_ctx* ctx, const stokes_fmm_plan* plan, int kernel, int64_t n_src, const double* src_xyz,
                    const double* density, const double* weight, const double* normal, int64_t n_trg,
                    const double* trg_xyz, double pref, const double* centre, double half_width, int32_t depth,
                    const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out, void* workspace,
                    size_t ws_bytes, void* stream) {
    const char* name = kernel ? "stokes_fmm_dl_eval" : "stokes_fmm_sl_eval";
    if (!ctx) return fail(STOKES_EINVAL, "ctx is NULL");
    int rc = fmm_check_sizes(plan, n_src, n_trg, depth);
    if (rc) return rc;
    if (stokes::fmm_plan_device(plan) != ctx->device) return fail(STOKES_EINVAL, "the plan was built on another device");
    if (!centre) return fail(STOKES_EINVAL, "centre (host, 3 doubles) is NULL");
    for (int c = 0; c < 3; ++c)
        if (!isfinite(centre[c])) return fail(STOKES_EINVAL, "centre must be finite");
    if (!(isfinite(half_width) && half_width > 0.0)) return fail(STOKES_EINVAL, "half_width must be finite and > 0");
    Parsed p;
    if ((rc = parse_common(excl, opts, n_src, n_trg, p))) return rc;
    int32_t ng = 0;
    if ((rc = fmm_groups(excl, &ng))) return rc;

    if ((rc = check_points(kernel, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz))) return rc;
    if (!arr_ok(vel_out, 3 * n_trg, 8)) return fail(STOKES_EINVAL, "vel_out must be non-NULL and 8-byte aligned");
    const size_t sb = (size_t)3 * n_src * 8, tb = (size_t)3 * n_trg * 8;
    if ((rc = check_no_alias(vel_out, tb, "vel_out",
                             {{src_xyz, sb}, {density, sb}, {weight, (size_t)n_src * 8}, {normal, kernel ? sb : 0},
                              {trg_xyz, tb}, {workspace, ws_bytes}})))
        return rc;
    size_t off_groups = 0;
    const size_t need = fmm_total_bytes(plan, kernel, n_src, n_trg, depth, ng, &off_groups);
    if ((rc = check_workspace(workspace, ws_bytes, need))) return rc;
    if (n_trg == 0) return STOKES_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(STOKES_EDEVICE, "cannot select the context's device");
    stokes::FmmInputs in{};
    in.n_src = n_src;
    in.n_trg = n_trg;
    in.src_xyz = src_xyz;
    in.density = density;
    in.weight = weight;
    in.normal = kernel ? normal : nullptr;
    in.trg_xyz = trg_xyz;
    for (int c = 0; c < 3; ++c) in.centre[c] = centre[c];
    in.half_width = half_width;
    in.depth = depth;
    in.pref = pref;
    in.accumulate = p.accumulate;
    in.mixed = p.precision == STOKES_MIXED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const stokes::KernelTimer timer = stokes::next_timer(ctx);
    if (timer.on()) (void)hipEventRecord(timer.start, st);
    hipError_t e = stokes::launch_fmm(plan, in, vel_out, workspace, st);
    if (e == hipSuccess && ng > 0 && n_src > 0) {
        // the same-group rule: take off each group's sum onto itself
        stokes::SumInputs g{};
        g.kernel = kernel;
        g.n_src = n_src;
        g.n_trg = n_trg;
        g.src_xyz = src_xyz;
        g.density = density;
        g.weight = weight;
        g.normal = kernel ? normal : nullptr;
        g.trg_xyz = trg_xyz;
        g.src_group = p.src_group;
        g.trg_group = p.trg_group;
        g.n_groups = ng;
        g.pref = kernel ? 6.0 / (8.0 * kPi) : pref;
        e = stokes::launch_same_group_subtract(g, vel_out, static_cast<char*>(workspace) + off_groups, st);
    }
    if (timer.on()) (void)hipEventRecord(timer.stop, st);
    return launch_status(e, name);
}

int stokes_fmm_sl_eval(stokes_ctx* ctx, const stokes_fmm_plan* plan, int64_t n_src, const double* src_xyz,
                       const double* density, const double* weight, int64_t n_trg, const double* trg_xyz,
                       double mu, const double* centre, double half_width, int32_t depth,
                       const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out, void* workspace,
                       size_t ws_bytes, void* stream) {
    if (!(isfinite(mu) && mu > 0.0)) return fail(STOKES_EINVAL, "mu must be finite and > 0");
    return fmm_eval(ctx, plan, STOKES_KERNEL_SL, n_src, src_xyz, density, weight, nullptr, n_trg, trg_xyz,
                    1.0 / (8.0 * kPi * mu), centre, half_width, depth, excl, opts, vel_out, workspace, ws_bytes,
                    stream);
}

int stokes_fmm_dl_eval(stokes_ctx* ctx, const stokes_fmm_plan* plan, int64_t n_src, const double* src_xyz,
                       const double* density, const double* weight, const double* normal, int64_t n_trg,
                       const double* trg_xyz, const double* centre, double half_width, int32_t depth,
                       const stokes_exclusion* excl, const stokes_opts* opts, double* vel_out, void* workspace,
                       size_t ws_bytes, void* stream) {
    return fmm_eval(ctx, plan, STOKES_KERNEL_DL, n_src, src_xyz, density, weight, normal, n_trg, trg_xyz,
                    1.0 / (8.0 * kPi), centre, half_width, depth, excl, opts, vel_out, workspace, ws_bytes, stream);
}

}  // extern "C"
