// Internal declarations of the spatial-hash candidate search (space-time
// bounding boxes, grid cells, Morton keys, radix sort, candidate pairs).  Not
// part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace stokes {

constexpr int kMortonBits = 21;                    // cell coordinates per axis < 2^21

// Per mesh m: min / max over points [ofs[m], ofs[m+1]) (clamped to [0, n_points];
// a decreasing pair is an empty mesh) of x0 and, when given, x1, moved out by
// inflate.  Empty meshes get lo = +inf, hi = -inf.
hipError_t launch_space_time_boxes(int32_t n_meshes, const int64_t* ofs, int64_t n_points, const double* x0,
                                   const double* x1, double inflate, double* lo, double* hi, hipStream_t stream);

// Workspace regions of one candidate search with room for max_entries
// (box, cell) entries.
struct CandidateLayout {
    int64_t max_entries = 0;
    int64_t sort_blocks = 0;
    size_t off_meta = 0, off_range = 0, off_count = 0, off_scan = 0, off_keys = 0, off_vals = 0, off_keys2 = 0,
           off_vals2 = 0, off_hist = 0, off_pcount = 0, total = 0;
};
CandidateLayout candidate_layout(int32_t n_boxes, int64_t max_entries);

// Host-visible summary of the first phase.
struct CandidateMeta {
    double origin[3];
    int64_t entries;          // (box, cell) entries
    int32_t max_cell;         // largest cell coordinate on any axis
    int32_t overflow;         // a cell coordinate >= 2^21, or a non-finite corner
};

// Phase 1: origin, cell ranges, entry counts and their prefix sums; copies the
// summary to *meta (blocks on the stream).
hipError_t candidate_phase1(int32_t n_boxes, const double* lo, const double* hi, double cell, char* ws,
                            const CandidateLayout& lay, CandidateMeta* meta, hipStream_t stream);

// Phase 2: entries, sort, pair counts; returns the number of candidate pairs
// (blocks on the stream).  Phase 3 writes the first `capacity` of them.
hipError_t candidate_phase2(int32_t n_boxes, const CandidateMeta& meta, char* ws, const CandidateLayout& lay,
                            int64_t* n_pairs, hipStream_t stream);
hipError_t candidate_phase3(int32_t n_boxes, const CandidateMeta& meta, char* ws, const CandidateLayout& lay,
                            int32_t* pairs, int64_t capacity, hipStream_t stream);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// keys (8 bits per pass), in place.  Workspace from sort_layout(max_n).
struct SortLayout {
    int64_t max_n = 0, blocks = 0;
    size_t off_keys2 = 0, off_vals2 = 0, off_hist = 0, off_scan = 0, off_total = 0, total = 0;
};
SortLayout sort_layout(int64_t max_n);
hipError_t radix_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, int bits, char* ws, const SortLayout& lay,
                            hipStream_t stream);

// Exclusive prefix sum of n int64 values (in may equal out); *total gets the
// sum.  scan_tmp holds scan_tmp_count(n) int64.
int64_t scan_tmp_count(int64_t n);
hipError_t exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* scan_tmp, int64_t* total,
                              hipStream_t stream);

}  // namespace stokes
