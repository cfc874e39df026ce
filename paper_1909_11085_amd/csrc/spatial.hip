// Spatial-hash candidate search on the GPU (Sec. 4, reusing steps a-c of the
// closest-point search of Sec. 3.3):
//
//   boxes        space-time bounding box per mesh: a workgroup per mesh, min /
//                max over its points at both time levels (exact, any order);
//   phase 1      grid origin (lowest valid corner), each box's integer cell
//                range floor((corner - origin) / H), its cell count, and the
//                exclusive prefix sum of the counts (two-level, exact);
//   phase 2      one (Morton key, box) entry per overlapped cell, an LSD radix
//                sort of the entries by key (8-bit digits, stable: wave ballots
//                rank equal digits in position order), then per entry the
//                number of later entries with the same key whose box pairs
//                with it for the first time in that cell; a prefix sum of
//                those counts;
//   phase 3      the pairs, written at their prefix-sum slots.
//
// A pair of boxes shares the cells of the intersection of their ranges; it is
// emitted only in the lowest of them, whose Morton key is the smallest since
// Morton order grows with each coordinate, so every pair appears exactly once.
// Output order: by that cell's key, then by the first box, then the second.
#include <float.h>
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "spatial.hpp"

namespace stokes {
namespace {

constexpr int kSpBlock = 256;
constexpr int kSpWaves = kSpBlock / kWave;
constexpr int kRadix = 256;                      // 8-bit digits; one digit per thread of a block
constexpr int kSortItems = 8;                     // most keys per thread of a sort workgroup
constexpr int kSortTile = kSpBlock * kSortItems;  // most keys per sort workgroup
constexpr int kScanItems = 8;
constexpr int kScanTile = kSpBlock * kScanItems;  // elements per scan workgroup
constexpr int64_t kSpMaxGrid = 1 << 16;
constexpr int kOriginBlocks = 64;                // workgroups of the origin reduction
static_assert(kSpBlock == kRadix, "one digit per thread");

unsigned sp_grid(int64_t units, int64_t per) {
    const int64_t b = (units + per - 1) / per;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kSpMaxGrid));
}

// NaN-propagating min / max (so a NaN coordinate makes the box invalid).
__device__ __forceinline__ double nmin(double a, double b) { return (b < a || b != b) ? b : a; }
__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

__global__ __launch_bounds__(kSpBlock) void boxes_kernel(int32_t n_meshes, const int64_t* __restrict__ ofs,
                                                         int64_t n, const double* __restrict__ x0,
                                                         const double* __restrict__ x1, double inflate,
                                                         double* __restrict__ lo, double* __restrict__ hi) {
    __shared__ double red[kSpWaves][6];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    for (int64_t m = blockIdx.x; m < n_meshes; m += gridDim.x) {      // uniform over the workgroup
        const int64_t a = std::min(std::max(ofs[m], (int64_t)0), n);
        const int64_t b = std::min(std::max(ofs[m + 1], (int64_t)0), n);
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = a + threadIdx.x; i < b; i += kSpBlock) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double v = x0[c * n + i];
                mn[c] = nmin(mn[c], v);
                mx[c] = nmax(mx[c], v);
                if (x1) {
                    const double w = x1[c * n + i];
                    mn[c] = nmin(mn[c], w);
                    mx[c] = nmax(mx[c], w);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            for (int o = kWave / 2; o >= 1; o >>= 1) {
                mn[c] = nmin(mn[c], __shfl_xor(mn[c], o));
                mx[c] = nmax(mx[c], __shfl_xor(mx[c], o));
            }
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                red[wave][c] = mn[c];
                red[wave][3 + c] = mx[c];
            }
        __syncthreads();
        if (threadIdx.x < 3) {
            const int c = threadIdx.x;
            double l = red[0][c], h = red[0][3 + c];
#pragma unroll
            for (int w = 1; w < kSpWaves; ++w) {
                l = nmin(l, red[w][c]);
                h = nmax(h, red[w][3 + c]);
            }
            lo[c * (int64_t)n_meshes + m] = b > a ? l - inflate : INFINITY;
            hi[c * (int64_t)n_meshes + m] = b > a ? h + inflate : -INFINITY;
        }
        __syncthreads();                          // red is reused by the next mesh
    }
}

// ------------------------------------------------------------------ phase 1
__device__ __forceinline__ bool box_valid(const double* lo, const double* hi, int32_t n, int64_t b) {
    return lo[b] <= hi[b] && lo[n + b] <= hi[n + b] && lo[2 * n + b] <= hi[2 * n + b];
}

// Stage 1 of the origin: per-workgroup minima of the valid boxes' lower
// corners (part[c * kOriginBlocks + block]); workgroup 0 also clears the
// summary's counters.
__global__ __launch_bounds__(kSpBlock) void origin_kernel(int32_t n, const double* __restrict__ lo,
                                                          const double* __restrict__ hi, double* __restrict__ part,
                                                          CandidateMeta* meta) {
    __shared__ double red[3][kSpBlock];
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    for (int64_t b = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; b < n; b += (int64_t)gridDim.x * kSpBlock)
        if (box_valid(lo, hi, n, b))
#pragma unroll
            for (int c = 0; c < 3; ++c) mn[c] = fmin(mn[c], lo[c * (int64_t)n + b]);
#pragma unroll
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = mn[c];
    __syncthreads();
    for (int o = kSpBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
#pragma unroll
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x < 3) part[threadIdx.x * kOriginBlocks + blockIdx.x] = red[threadIdx.x][0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) meta->origin[c] = 0.0;
        meta->entries = 0;
        meta->max_cell = 0;
        meta->overflow = 0;
    }
}

// Cell range (clo in rows 0..2, chi in rows 3..5) and cell count per box.
// Each workgroup first finishes the origin from the stage-1 minima (the
// lowest valid corner, 0 when there is none); workgroup 0 records it.
__global__ __launch_bounds__(kSpBlock) void cells_kernel(int32_t n, const double* __restrict__ lo,
                                                         const double* __restrict__ hi, double H,
                                                         const double* __restrict__ part, CandidateMeta* meta,
                                                         int32_t* __restrict__ range, int64_t* __restrict__ count) {
    __shared__ double s_o[3];
    if (threadIdx.x < 3) {
        double v = INFINITY;
        for (int g = 0; g < kOriginBlocks; ++g) v = fmin(v, part[threadIdx.x * kOriginBlocks + g]);
        s_o[threadIdx.x] = v < INFINITY ? v : 0.0;
        if (blockIdx.x == 0) meta->origin[threadIdx.x] = s_o[threadIdx.x];
    }
    __syncthreads();
    const double o[3] = {s_o[0], s_o[1], s_o[2]};
    for (int64_t b = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; b < n; b += (int64_t)gridDim.x * kSpBlock) {
        int64_t cnt = 0;
        int32_t r[6] = {1, 1, 1, 0, 0, 0};
        if (box_valid(lo, hi, n, b)) {
            bool ok = true;
            int32_t top = 0;
            cnt = 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double a = floor((lo[c * (int64_t)n + b] - o[c]) / H);
                const double e = floor((hi[c * (int64_t)n + b] - o[c]) / H);
                ok = ok && a >= 0.0 && e < (double)(1 << kMortonBits);     // false for NaN and infinities
                if (ok) {
                    r[c] = (int32_t)a;
                    r[3 + c] = (int32_t)e;
                    cnt *= (int64_t)(r[3 + c] - r[c] + 1);
                    top = std::max(top, r[3 + c]);
                }
            }
            if (!ok) {
                atomicOr(&meta->overflow, 1);
                cnt = 0;
                r[0] = r[1] = r[2] = 1;
                r[3] = r[4] = r[5] = 0;
            } else {
                atomicMax(&meta->max_cell, top);
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) range[c * (int64_t)n + b] = r[c];
        count[b] = cnt;
    }
}

// Exclusive prefix sum of int64 values, in three kernels: per-workgroup sums,
// a sequential scan of those sums (one thread), per-workgroup scans plus their
// offsets.  Exact, so the order does not matter for the result.
__global__ __launch_bounds__(kSpBlock) void scan_sums_kernel(const int64_t* __restrict__ in, int64_t n,
                                                             int64_t* __restrict__ sums) {
    __shared__ int64_t red[kSpBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) s += in[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kSpBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void scan_top_kernel(int64_t* sums, int64_t nb, int64_t* total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t v = sums[b];
        sums[b] = acc;
        acc += v;
    }
    *total = acc;
}

__global__ __launch_bounds__(kSpBlock) void scan_final_kernel(const int64_t* __restrict__ in, int64_t n,
                                                              const int64_t* __restrict__ sums,
                                                              int64_t* __restrict__ out) {
    __shared__ int64_t pre[kSpBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    pre[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kSpBlock; o <<= 1) {          // inclusive Hillis-Steele scan of the thread sums
        const int64_t add = (int)threadIdx.x >= o ? pre[threadIdx.x - o] : 0;
        __syncthreads();
        pre[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t acc = sums[blockIdx.x] + pre[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) out[i] = acc;
        acc += v[k];
    }
}

// scan_tmp: (n + kScanTile - 1) / kScanTile int64 sums.
hipError_t exclusive_scan(const int64_t* in, int64_t n, int64_t* out, int64_t* scan_tmp, int64_t* total,
                          hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(kSpBlock), 0, st, in, n, scan_tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kWave), 0, st, scan_tmp, nb, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scan_final_kernel, dim3((unsigned)nb), dim3(kSpBlock), 0, st, in, n, scan_tmp, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ phase 2
// 21-bit Morton interleave by the standard mask-and-shift spreading.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}
__device__ __forceinline__ uint64_t morton(int32_t x, int32_t y, int32_t z) {
    return spread3((uint64_t)x) | spread3((uint64_t)y) << 1 | spread3((uint64_t)z) << 2;
}

__global__ __launch_bounds__(kSpBlock) void emit_kernel(int32_t n, const int32_t* __restrict__ range,
                                                        const int64_t* __restrict__ offs,
                                                        uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    for (int64_t b = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; b < n; b += (int64_t)gridDim.x * kSpBlock) {
        const int32_t x0 = range[b], y0 = range[n + b], z0 = range[2 * (int64_t)n + b];
        const int32_t x1 = range[3 * (int64_t)n + b], y1 = range[4 * (int64_t)n + b], z1 = range[5 * (int64_t)n + b];
        int64_t o = offs[b];
        for (int32_t x = x0; x <= x1; ++x)
            for (int32_t y = y0; y <= y1; ++y)
                for (int32_t z = z0; z <= z1; ++z) {
                    keys[o] = morton(x, y, z);
                    vals[o] = (int32_t)b;
                    ++o;
                }
    }
}

// Digit counts of one sort workgroup's tile, digit-major: hist[d * nb + block].
__global__ __launch_bounds__(kSpBlock) void rs_hist_kernel(const uint64_t* __restrict__ keys, int64_t E,
                                                           int shift, int items, int64_t* __restrict__ hist,
                                                           int64_t nb) {
    __shared__ int cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSpBlock * items;
    for (int k = 0; k < items; ++k) {
        const int64_t i = base + (int64_t)k * kSpBlock + threadIdx.x;
        if (i < E) atomicAdd(&cnt[(int)((keys[i] >> shift) & 0xff)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: the tile is taken in chunks of 256 in position order; inside
// a chunk each key's rank among equal digits comes from wave ballots (lanes
// below it with the same digit) plus the counts of the waves before it.
__global__ __launch_bounds__(kSpBlock) void rs_scatter_kernel(const uint64_t* __restrict__ keys,
                                                              const int32_t* __restrict__ vals, int64_t E,
                                                              int shift, int items, const int64_t* __restrict__ hoff,
                                                              int64_t nb, uint64_t* __restrict__ keys_out,
                                                              int32_t* __restrict__ vals_out) {
    __shared__ int64_t run[kRadix];
    __shared__ int wcnt[kSpWaves][kRadix];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    run[tid] = hoff[(int64_t)tid * nb + blockIdx.x];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int64_t base = (int64_t)blockIdx.x * kSpBlock * items;
    for (int k = 0; k < items; ++k) {
#pragma unroll
        for (int w = 0; w < kSpWaves; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)k * kSpBlock + tid;
        const bool valid = i < E;
        const uint64_t key = valid ? keys[i] : 0ull;
        const int32_t val = valid ? vals[i] : 0;
        const int d = (int)((key >> shift) & 0xff);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t set = __ballot((d >> bit) & 1);
            peers &= ((d >> bit) & 1) ? set : ~set;
        }
        const int rank = __popcll(peers & below);
        const int group = __popcll(peers);
        if (valid && rank == group - 1) wcnt[wave][d] = group;     // one writer per (wave, digit)
        __syncthreads();
        int pre[kSpWaves];
        int acc = 0;
#pragma unroll
        for (int w = 0; w < kSpWaves; ++w) {
            pre[w] = acc;
            acc += wcnt[w][tid];
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kSpWaves; ++w) wcnt[w][tid] = pre[w];
        __syncthreads();
        if (valid) {
            const int64_t pos = run[d] + wcnt[wave][d] + rank;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        run[tid] += acc;
        __syncthreads();
    }
}

// Per sorted entry e (box a, cell key k): later entries with the same key whose
// box b has the cell k as the lowest cell of the two ranges' intersection.
template <bool EMIT>
__global__ __launch_bounds__(kSpBlock) void pairs_kernel(int64_t E, const uint64_t* __restrict__ keys,
                                                         const int32_t* __restrict__ vals, int32_t n,
                                                         const int32_t* __restrict__ range,
                                                         int64_t* __restrict__ counts,
                                                         const int64_t* __restrict__ offs,
                                                         int32_t* __restrict__ pairs, int64_t capacity) {
    for (int64_t e = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; e < E; e += (int64_t)gridDim.x * kSpBlock) {
        const uint64_t k = keys[e];
        const int32_t a = vals[e];
        const int32_t ax = range[a], ay = range[n + a], az = range[2 * (int64_t)n + a];
        int64_t cnt = 0, slot = EMIT ? offs[e] : 0;
        for (int64_t f = e + 1; f < E && keys[f] == k; ++f) {
            const int32_t b = vals[f];
            const int32_t bx = range[b], by = range[n + b], bz = range[2 * (int64_t)n + b];
            if (morton(std::max(ax, bx), std::max(ay, by), std::max(az, bz)) != k) continue;
            if (EMIT) {
                if (slot < capacity) {
                    pairs[slot] = a;
                    pairs[capacity + slot] = b;
                }
                ++slot;
            } else {
                ++cnt;
            }
        }
        if (!EMIT) counts[e] = cnt;
    }
}

}  // namespace

hipError_t launch_space_time_boxes(int32_t n_meshes, const int64_t* ofs, int64_t n_points, const double* x0,
                                   const double* x1, double inflate, double* lo, double* hi, hipStream_t stream) {
    if (n_meshes <= 0) return hipSuccess;
    hipLaunchKernelGGL(boxes_kernel, dim3(sp_grid(n_meshes, 1)), dim3(kSpBlock), 0, stream, n_meshes, ofs,
                       n_points, x0, x1, inflate, lo, hi);
    return hipGetLastError();
}

CandidateLayout candidate_layout(int32_t n_boxes, int64_t max_entries) {
    CandidateLayout L;
    L.max_entries = max_entries;
    L.sort_blocks = std::max<int64_t>(1, (max_entries + kSortTile - 1) / kSortTile);
    const int64_t nscan = std::max<int64_t>({(int64_t)n_boxes, max_entries, kRadix * L.sort_blocks}) + 1;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t nb = (size_t)std::max<int32_t>(n_boxes, 1), ne = (size_t)std::max<int64_t>(max_entries, 1);
    L.off_meta = take(sizeof(CandidateMeta) + 2 * sizeof(int64_t) + 3 * kOriginBlocks * sizeof(double));
    L.off_range = take(6 * nb * sizeof(int32_t));
    L.off_count = take(2 * (nb + 1) * sizeof(int64_t));                // counts, then offsets
    L.off_scan = take(((size_t)nscan / kScanTile + 2) * sizeof(int64_t));
    L.off_keys = take(ne * sizeof(uint64_t));
    L.off_vals = take(ne * sizeof(int32_t));
    L.off_keys2 = take(ne * sizeof(uint64_t));
    L.off_vals2 = take(ne * sizeof(int32_t));
    L.off_hist = take(2 * (size_t)kRadix * L.sort_blocks * sizeof(int64_t));   // counts, then offsets
    L.off_pcount = take(2 * ne * sizeof(int64_t));                     // pair counts, then offsets
    L.total = off;
    return L;
}

hipError_t candidate_phase1(int32_t n_boxes, const double* lo, const double* hi, double cell, char* ws,
                            const CandidateLayout& L, CandidateMeta* meta, hipStream_t st) {
    CandidateMeta* dmeta = reinterpret_cast<CandidateMeta*>(ws + L.off_meta);
    int32_t* range = reinterpret_cast<int32_t*>(ws + L.off_range);
    int64_t* count = reinterpret_cast<int64_t*>(ws + L.off_count);
    int64_t* offs = count + (n_boxes + 1);
    int64_t* tmp = reinterpret_cast<int64_t*>(ws + L.off_scan);
    double* part = reinterpret_cast<double*>(ws + L.off_meta + sizeof(CandidateMeta) + 2 * sizeof(int64_t));
    hipLaunchKernelGGL(origin_kernel, dim3(kOriginBlocks), dim3(kSpBlock), 0, st, n_boxes, lo, hi, part, dmeta);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && n_boxes > 0) {
        hipLaunchKernelGGL(cells_kernel, dim3(sp_grid(n_boxes, kSpBlock)), dim3(kSpBlock), 0, st, n_boxes, lo, hi,
                           cell, part, dmeta, range, count);
        e = hipGetLastError();
        if (e == hipSuccess) e = exclusive_scan(count, n_boxes, offs, tmp, &dmeta->entries, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(meta, dmeta, sizeof(CandidateMeta), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// Radix passes for the keys of this search, and the buffers that hold the
// sorted entries after them (the sort ping-pongs between the two).
static int sort_passes(const CandidateMeta& meta) {
    int bits = 0;
    while (bits < kMortonBits && (meta.max_cell >> bits) != 0) ++bits;
    return std::max(1, (3 * bits + 7) / 8);
}

hipError_t candidate_phase2(int32_t n_boxes, const CandidateMeta& meta, char* ws, const CandidateLayout& L,
                            int64_t* n_pairs, hipStream_t st) {
    *n_pairs = 0;
    const int64_t E = meta.entries;
    if (E <= 0) return hipSuccess;
    int32_t* range = reinterpret_cast<int32_t*>(ws + L.off_range);
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.off_count) + (n_boxes + 1);
    int64_t* tmp = reinterpret_cast<int64_t*>(ws + L.off_scan);
    uint64_t* keys = reinterpret_cast<uint64_t*>(ws + L.off_keys);
    int32_t* vals = reinterpret_cast<int32_t*>(ws + L.off_vals);
    uint64_t* keys2 = reinterpret_cast<uint64_t*>(ws + L.off_keys2);
    int32_t* vals2 = reinterpret_cast<int32_t*>(ws + L.off_vals2);
    int64_t* hist = reinterpret_cast<int64_t*>(ws + L.off_hist);
    int64_t* pcount = reinterpret_cast<int64_t*>(ws + L.off_pcount);
    int64_t* total = reinterpret_cast<int64_t*>(ws + L.off_meta + sizeof(CandidateMeta));
    hipLaunchKernelGGL(emit_kernel, dim3(sp_grid(n_boxes, kSpBlock)), dim3(kSpBlock), 0, st, n_boxes, range, offs,
                       keys, vals);
    hipError_t e = hipGetLastError();
    const int passes = sort_passes(meta);
    // the fewest keys per thread (so the most workgroups) that the histogram
    // space, sized for kSortTile keys per workgroup, allows
    const int items = (int)std::min<int64_t>(
        kSortItems, std::max<int64_t>(1, (E + (int64_t)kSpBlock * L.sort_blocks - 1) / ((int64_t)kSpBlock * L.sort_blocks)));
    const int64_t nb = (E + (int64_t)kSpBlock * items - 1) / ((int64_t)kSpBlock * items);
    int64_t* hoff = hist + (int64_t)kRadix * nb;
    for (int p = 0; p < passes && e == hipSuccess; ++p) {
        hipLaunchKernelGGL(rs_hist_kernel, dim3((unsigned)nb), dim3(kSpBlock), 0, st, keys, E, 8 * p, items, hist,
                           nb);
        e = hipGetLastError();
        if (e == hipSuccess) e = exclusive_scan(hist, (int64_t)kRadix * nb, hoff, tmp, total, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(rs_scatter_kernel, dim3((unsigned)nb), dim3(kSpBlock), 0, st, keys, vals, E, 8 * p,
                               items, hoff, nb, keys2, vals2);
            e = hipGetLastError();
        }
        std::swap(keys, keys2);
        std::swap(vals, vals2);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pairs_kernel<false>, dim3(sp_grid(E, kSpBlock)), dim3(kSpBlock), 0, st, E, keys, vals,
                           n_boxes, range, pcount, nullptr, nullptr, (int64_t)0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = exclusive_scan(pcount, E, pcount + E, tmp, total, st);
    if (e == hipSuccess) e = hipMemcpyAsync(n_pairs, total, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

hipError_t candidate_phase3(int32_t n_boxes, const CandidateMeta& meta, char* ws, const CandidateLayout& L,
                            int32_t* pairs, int64_t capacity, hipStream_t st) {
    const int64_t E = meta.entries;
    if (E <= 0 || capacity <= 0) return hipSuccess;
    const bool second = sort_passes(meta) & 1;         // the last pass wrote the second buffers
    const uint64_t* keys = reinterpret_cast<const uint64_t*>(ws + (second ? L.off_keys2 : L.off_keys));
    const int32_t* vals = reinterpret_cast<const int32_t*>(ws + (second ? L.off_vals2 : L.off_vals));
    const int32_t* range = reinterpret_cast<const int32_t*>(ws + L.off_range);
    const int64_t* poffs = reinterpret_cast<const int64_t*>(ws + L.off_pcount) + E;
    hipLaunchKernelGGL(pairs_kernel<true>, dim3(sp_grid(E, kSpBlock)), dim3(kSpBlock), 0, st, E, keys, vals, n_boxes,
                       range, nullptr, poffs, pairs, capacity);
    return hipGetLastError();
}

SortLayout sort_layout(int64_t max_n) {
    SortLayout L;
    L.max_n = max_n;
    L.blocks = std::max<int64_t>(1, (max_n + kSortTile - 1) / kSortTile);
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t n = (size_t)std::max<int64_t>(max_n, 1);
    L.off_keys2 = take(n * sizeof(uint64_t));
    L.off_vals2 = take(n * sizeof(int32_t));
    L.off_hist = take(2 * (size_t)kRadix * L.blocks * sizeof(int64_t));
    L.off_scan = take(((size_t)kRadix * L.blocks / kScanTile + 2) * sizeof(int64_t));
    L.off_total = take(sizeof(int64_t));
    L.total = off;
    return L;
}

namespace {
__global__ __launch_bounds__(kSpBlock) void copy_pairs_kernel(const uint64_t* __restrict__ ks,
                                                              const int32_t* __restrict__ vs, int64_t n,
                                                              uint64_t* __restrict__ kd, int32_t* __restrict__ vd) {
    for (int64_t i = (int64_t)blockIdx.x * kSpBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSpBlock) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}
}  // namespace

hipError_t radix_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, int bits, char* ws, const SortLayout& L,
                            hipStream_t st) {
    if (n <= 1) return hipSuccess;
    uint64_t* k2 = reinterpret_cast<uint64_t*>(ws + L.off_keys2);
    int32_t* v2 = reinterpret_cast<int32_t*>(ws + L.off_vals2);
    int64_t* hist = reinterpret_cast<int64_t*>(ws + L.off_hist);
    int64_t* tmp = reinterpret_cast<int64_t*>(ws + L.off_scan);
    int64_t* total = reinterpret_cast<int64_t*>(ws + L.off_total);
    const int passes = std::max(1, (bits + 7) / 8);
    const int items = (int)std::min<int64_t>(
        kSortItems, std::max<int64_t>(1, (n + (int64_t)kSpBlock * L.blocks - 1) / ((int64_t)kSpBlock * L.blocks)));
    const int64_t nb = (n + (int64_t)kSpBlock * items - 1) / ((int64_t)kSpBlock * items);
    int64_t* hoff = hist + (int64_t)kRadix * nb;
    uint64_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes && e == hipSuccess; ++p) {
        hipLaunchKernelGGL(rs_hist_kernel, dim3((unsigned)nb), dim3(kSpBlock), 0, st, ka, n, 8 * p, items, hist, nb);
        e = hipGetLastError();
        if (e == hipSuccess) e = exclusive_scan(hist, (int64_t)kRadix * nb, hoff, tmp, total, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(rs_scatter_kernel, dim3((unsigned)nb), dim3(kSpBlock), 0, st, ka, va, n, 8 * p, items,
                               hoff, nb, kb, vb);
            e = hipGetLastError();
        }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (e == hipSuccess && ka != keys) {          // odd pass count: the result sits in the second buffers
        hipLaunchKernelGGL(copy_pairs_kernel, dim3(sp_grid(n, kSpBlock)), dim3(kSpBlock), 0, st, ka, va, n, keys,
                           vals);
        e = hipGetLastError();
    }
    return e;
}

int64_t scan_tmp_count(int64_t n) { return std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile) + 1; }

hipError_t exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* scan_tmp, int64_t* total,
                              hipStream_t stream) {
    return exclusive_scan(in, n, out, scan_tmp, total, stream);
}

}  // namespace stokes
