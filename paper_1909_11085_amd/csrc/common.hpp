// Internal declarations shared by the HIP translation units of the Stokes
// kernel-sum library (gfx950).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace stokes {

constexpr int kWave = 64;        // CDNA wavefront
constexpr int kBlock = 256;      // 4 waves per workgroup
constexpr int kSub = 64;         // sources per sub-tile (unit of the far/near box test)
constexpr int kTile = 256;       // sources staged in LDS per step (4 sub-tiles)

// Padding sources sit this far out with zero strength; inputs must stay well
// inside |coordinate| < 1e100 so that padding pairs stay finite and add 0.
constexpr double kPadPos = 1.0e150;
constexpr float kPadOff = 1.0e18f;

// Per-sub-tile summary written by the source prep kernel.
struct alignas(16) SubMeta {
    double lo[3], hi[3];   // bounding box of the sub-tile's real sources
    double ctr[3];         // box centre; mixed-precision offsets are relative to it
    double rnear;          // largest near radius (mixed) in the sub-tile, else 0
    int32_t gmin, gmax;    // group id range of the sub-tile
    int32_t count;         // real sources in the sub-tile (0..64)
    int32_t pad;
};

// Packed source records (one per source, padded to a multiple of kTile).
// Strength q = w * density is formed by the prep kernel.
struct alignas(16) SrcSL64 { double x, y, z, qx, qy, qz; };                       // 48 B
struct alignas(16) SrcDL64 { double x, y, z, qx, qy, qz, nx, ny, nz, pad; };      // 80 B
// Direct FP64 single layer: positions stored doubled (2y, exact) and both q and
// 4q, so that the pair needs no constant multiplies (see direct.hip).
struct alignas(16) SrcSL64x { double x, y, z, qx, qy, qz, q4x, q4y, q4z, pad; };  // 80 B
struct alignas(16) SrcSL32 { float ox, oy, oz, qx, qy, qz, t2; int32_t g; };      // 32 B
struct alignas(16) SrcDL32 { float ox, oy, oz, qx, qy, qz, nx, ny, nz, t2; int32_t g; float pad; }; // 48 B

template <int KT, int MIXED> struct SrcRec;
template <> struct SrcRec<0, 0> { using type = SrcSL64x; };
template <> struct SrcRec<1, 0> { using type = SrcDL64; };
template <> struct SrcRec<0, 1> { using type = SrcSL32; };
template <> struct SrcRec<1, 1> { using type = SrcDL32; };

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Inputs of a direct (all-pairs) sum, in caller layout.
struct SumInputs {
    int kernel;                  // 0 = single layer, 1 = double layer
    int mixed;                   // 0 = FP64, 1 = mixed
    int64_t n_src, n_trg;
    const double* src_xyz;       // (3, n_src)
    const double* density;       // (3, n_src)
    const double* weight;        // (n_src)
    const double* normal;        // (3, n_src), DL only
    const double* trg_xyz;       // (3, n_trg)
    int excl;                    // 0 none, 1 same group
    const int32_t* src_group;    // may be null when excl == 0 and no near rule
    const int32_t* trg_group;
    const double* group_h;       // mixed near rule, may be null
    int32_t n_groups;
    double near_frac;
    double pref;                 // 1/(8 pi mu) or 6/(8 pi)
    // test-only: when set, the mixed direct and leaf-to-leaf kernels add, for
    // every pair they take, its class code into pair_class[t * n_src + s]
    int32_t* pair_class;
    // leaf-to-leaf sums: when set, target t's result goes to output column
    // trg_perm[t] (points sorted by an internal caller); a null weight is 1
    const int32_t* trg_perm;
    // leaf-to-leaf kernel-gradient sums (kernel = 2): per-target vector (3, n_trg)
    const double* trg_vec;
    const double* trg_vec2;    // a second vector per target (leaf-to-leaf adjoint sums, kernel 5)
};

// class codes of pair_class (one pair taken once holds exactly one of them)
constexpr int32_t kPairF32 = 1;        // float32 pair
constexpr int32_t kPairF64 = 1 << 8;   // float64 near pair
constexpr int32_t kPairSkip = 1 << 16; // excluded: same group, or zero distance

// Launch shape of a direct sum; a pure function of sizes and options so that
// the workspace query and the evaluation agree.
struct DirectPlan {
    int T;                       // targets per lane
    int64_t n_src_pad;           // sources padded to kTile
    int64_t n_sub;               // n_src_pad / kSub
    int64_t chunks;              // n_src_pad / kTile
    int64_t blocks_x;            // target blocks of kBlock * T targets
    int64_t units;               // blocks_x * chunks
    int64_t grid;                // workgroups (resident count, at most units)
    size_t off_src, off_grp, off_meta, off_part, off_near, off_flags, total;
};

// Workgroups of a direct-sum kernel that fit on one compute unit at once.
int direct_blocks_per_cu(int kernel, int mixed);

// resident_blocks: workgroups resident on the whole device; forced_grid > 0
// overrides it (tests).
DirectPlan plan_direct(int kernel, int mixed, int64_t n_src, int64_t n_trg, int resident_blocks,
                       int forced_grid);

// Optional event pair recorded around a call's main summation kernel(s).
struct KernelTimer {
    hipEvent_t start = nullptr, stop = nullptr;
    bool on() const { return start != nullptr; }
};

// Launches prep + sum (+ reduction) on `stream`.  Returns a hipError_t.
hipError_t launch_direct(const SumInputs& in, const DirectPlan& p, double* out, int accumulate,
                         void* workspace, hipStream_t stream, const KernelTimer& timer);

// Packs n_pad (a multiple of kBlock) source records, padding beyond n_src, and
// the per-64-source summaries (the direct sums' prep kernel).
hipError_t launch_prep(const SumInputs& in, int64_t n_pad, void* rec, void* aux, SubMeta* meta,
                       hipStream_t stream);

// Each-pair-once float64 single-layer sums over a shared point set (sources
// are the targets, one group array): every unordered pair is evaluated once
// for both of its points, for the forward sum (adjoint = 0) or for the
// adjoint's dL/df and total dL/dx (adjoint = 1).  Launch shape and
// workspace, a pure function of n.
struct SymPlan {
    int T;                       // 64-point tiles per wave (rows per lane)
    int64_t n_pad;               // points padded to a whole row block
    int64_t NT;                  // 64-point tiles
    int64_t NW;                  // row blocks (4 T tiles each)
    int64_t units;               // (row block, column tile) units of the triangle
    int64_t grid;                // workgroups
    size_t off_rec, off_aux, off_meta, off_row, off_col, total;
};
int sym_blocks_per_cu(int adjoint);
SymPlan plan_sym(int adjoint, int64_t n, int resident_blocks, int forced_grid);
hipError_t launch_sym(const SumInputs& in, const SymPlan& p, double* out, int accumulate, void* workspace,
                      hipStream_t stream, const KernelTimer& timer);
// grad_density (dL/df) and grad_xyz (the total dL/dx) may each be null.
hipError_t launch_sym_vjp(const SumInputs& in, const SymPlan& p, const double* grad_vel, double* grad_density,
                          double* grad_xyz, int accumulate, void* workspace, hipStream_t stream,
                          const KernelTimer& timer);

// Writes zeros into n doubles (used for empty source sets).
hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t stream);

}  // namespace stokes
