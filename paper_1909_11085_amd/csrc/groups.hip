// Same-group correction of a sum over all pairs: the FMM sums every pair
// (Sec. 3.1, "Far evaluation"), while the paper's sums skip the pairs of a
// cell with itself (Sec. 2.2, step 1(d), j != i).  The pairs a group holds
// with itself are summed exactly here and taken off the all-pairs result:
//   out(:, n) -= pref * sum over sources m of n's group, rho > 0, of K(x_n - y_m) q_m.
// What stays is the sum over pairs of different groups, up to the FMM's own
// error on the same-group pairs it approximated.
//
// Steps (one stream, no host round trip): group ids as sort keys (an id
// outside [0, n_groups) flags the call), a stable radix sort of sources and
// of targets by group, the group offsets, the sorted points gathered, the
// leaf-to-leaf kernel with every group a leaf listing only itself (float64),
// and the result subtracted in the caller's target order.  The sorts are
// stable and every sum runs in a fixed order: deterministic.
#include <algorithm>

#include "groups.hpp"
#include "p2p.hpp"
#include "spatial.hpp"

namespace stokes {
namespace {

constexpr int kGThreads = 256;

unsigned grid_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kGThreads - 1) / kGThreads, 8192));
}

int key_bits(int32_t n_groups) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n_groups) ++b;
    return b;
}

struct GroupLayout {
    SortLayout sort;
    size_t off_status, off_skeys, off_svals, off_tkeys, off_tvals, off_sofs, off_tofs, off_uofs, off_ul, off_sx,
        off_sd, off_sw, off_sn, off_tx, off_u, off_sort, off_p2p, total;
};

GroupLayout group_layout(int kernel, int64_t ns, int64_t nt, int32_t ng) {
    GroupLayout l{};
    const int64_t nmax = std::max<int64_t>(std::max(ns, nt), 1);
    l.sort = sort_layout(nmax);
    size_t off = 0;
    auto take = [&](size_t& o, size_t bytes) {
        o = off;
        off = align_up(off + std::max<size_t>(bytes, 8), 256);
    };
    take(l.off_status, sizeof(int32_t));
    take(l.off_skeys, (size_t)ns * 8);
    take(l.off_svals, (size_t)ns * 4);
    take(l.off_tkeys, (size_t)nt * 8);
    take(l.off_tvals, (size_t)nt * 4);
    take(l.off_sofs, (size_t)(ng + 1) * 8);
    take(l.off_tofs, (size_t)(ng + 1) * 8);
    take(l.off_uofs, (size_t)(ng + 1) * 8);
    take(l.off_ul, (size_t)ng * 4);
    take(l.off_sx, (size_t)ns * 24);
    take(l.off_sd, (size_t)ns * 24);
    take(l.off_sw, (size_t)ns * 8);
    take(l.off_sn, kernel ? (size_t)ns * 24 : 8);
    take(l.off_tx, (size_t)nt * 24);
    take(l.off_u, (size_t)nt * 24);
    take(l.off_sort, l.sort.total);
    take(l.off_p2p, p2p_workspace_bytes(kernel, 0, ns, nt, ng));
    l.total = off;
    return l;
}

__global__ __launch_bounds__(kGThreads) void g_clear(int32_t* status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

// keys = group ids (0 for an id outside [0, ng), which also flags the call)
__global__ __launch_bounds__(kGThreads) void g_keys(const int32_t* __restrict__ grp, int64_t n, int32_t ng,
                                                    uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                    int32_t* __restrict__ status) {
    for (int64_t i = (int64_t)blockIdx.x * kGThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kGThreads) {
        const int32_t g = grp[i];
        const bool ok = g >= 0 && g < ng;
        if (!ok) atomicOr(status, 1);
        keys[i] = ok ? (uint64_t)g : 0;
        vals[i] = (int32_t)i;
    }
}

// ofs[g] = first sorted position whose key is >= g, for g in [0, ng]
__global__ __launch_bounds__(kGThreads) void g_offsets(const uint64_t* __restrict__ keys, int64_t n, int32_t ng,
                                                       int64_t* __restrict__ ofs) {
    for (int64_t i = (int64_t)blockIdx.x * kGThreads + threadIdx.x; i <= n; i += (int64_t)gridDim.x * kGThreads) {
        const int64_t kp = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t kc = i == n ? (int64_t)ng : (int64_t)keys[i];
        for (int64_t g = kp + 1; g <= kc; ++g) ofs[g] = i;
    }
}

// every group lists itself
__global__ __launch_bounds__(kGThreads) void g_self_lists(int32_t ng, int64_t* __restrict__ uofs,
                                                          int32_t* __restrict__ ul) {
    for (int64_t g = (int64_t)blockIdx.x * kGThreads + threadIdx.x; g <= ng; g += (int64_t)gridDim.x * kGThreads) {
        uofs[g] = g;
        if (g < ng) ul[g] = (int32_t)g;
    }
}

// dst(:, i) = src(:, perm[i]) for c components of a (c, n) array
__global__ __launch_bounds__(kGThreads) void g_gather(const double* __restrict__ src, const int32_t* __restrict__ perm,
                                                      int64_t n, int c, double* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * kGThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kGThreads) {
        const int64_t m = perm[i];
        for (int q = 0; q < c; ++q) dst[q * n + i] = src[q * n + m];
    }
}

// out(:, perm[i]) -= u(:, i); a flagged call makes every component NaN
__global__ __launch_bounds__(kGThreads) void g_subtract(const double* __restrict__ u, const int32_t* __restrict__ perm,
                                                        int64_t n, const int32_t* __restrict__ status,
                                                        double* __restrict__ out) {
    const bool bad = *status != 0;
    for (int64_t i = (int64_t)blockIdx.x * kGThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kGThreads) {
        const int64_t o = perm[i];
        for (int q = 0; q < 3; ++q)
            out[q * n + o] = bad ? __builtin_nan("") : out[q * n + o] - u[q * n + i];
    }
}

}  // namespace

size_t same_group_workspace_bytes(int kernel, int64_t n_src, int64_t n_trg, int32_t n_groups) {
    if (n_src <= 0 || n_trg <= 0 || n_groups <= 0) return 0;
    return group_layout(kernel, n_src, n_trg, n_groups).total;
}

hipError_t launch_same_group_subtract(const SumInputs& in, double* out, void* ws, hipStream_t st) {
    const int64_t ns = in.n_src, nt = in.n_trg;
    const int32_t ng = in.n_groups;
    if (ns <= 0 || nt <= 0) return hipSuccess;
    const GroupLayout l = group_layout(in.kernel, ns, nt, ng);
    char* base = static_cast<char*>(ws);
    auto at = [&](size_t o) { return static_cast<void*>(base + o); };
    int32_t* status = static_cast<int32_t*>(at(l.off_status));
    uint64_t* skeys = static_cast<uint64_t*>(at(l.off_skeys));
    int32_t* svals = static_cast<int32_t*>(at(l.off_svals));
    uint64_t* tkeys = static_cast<uint64_t*>(at(l.off_tkeys));
    int32_t* tvals = static_cast<int32_t*>(at(l.off_tvals));
    int64_t* sofs = static_cast<int64_t*>(at(l.off_sofs));
    int64_t* tofs = static_cast<int64_t*>(at(l.off_tofs));
    int64_t* uofs = static_cast<int64_t*>(at(l.off_uofs));
    int32_t* ul = static_cast<int32_t*>(at(l.off_ul));
    double* sx = static_cast<double*>(at(l.off_sx));
    double* sd = static_cast<double*>(at(l.off_sd));
    double* sw = static_cast<double*>(at(l.off_sw));
    double* sn = static_cast<double*>(at(l.off_sn));
    double* tx = static_cast<double*>(at(l.off_tx));
    double* u = static_cast<double*>(at(l.off_u));
    char* sort_ws = base + l.off_sort;
    hipError_t e;
    auto chk = [&]() { return (e = hipGetLastError()) == hipSuccess; };
    const int bits = key_bits(ng);

    g_clear<<<1, kGThreads, 0, st>>>(status);
    if (!chk()) return e;
    g_keys<<<grid_for(ns), kGThreads, 0, st>>>(in.src_group, ns, ng, skeys, svals, status);
    if (!chk()) return e;
    g_keys<<<grid_for(nt), kGThreads, 0, st>>>(in.trg_group, nt, ng, tkeys, tvals, status);
    if (!chk()) return e;
    if ((e = radix_sort_pairs(skeys, svals, ns, bits, sort_ws, l.sort, st)) != hipSuccess) return e;
    if ((e = radix_sort_pairs(tkeys, tvals, nt, bits, sort_ws, l.sort, st)) != hipSuccess) return e;
    g_offsets<<<grid_for(ns + 1), kGThreads, 0, st>>>(skeys, ns, ng, sofs);
    if (!chk()) return e;
    g_offsets<<<grid_for(nt + 1), kGThreads, 0, st>>>(tkeys, nt, ng, tofs);
    if (!chk()) return e;
    g_self_lists<<<grid_for((int64_t)ng + 1), kGThreads, 0, st>>>(ng, uofs, ul);
    if (!chk()) return e;
    g_gather<<<grid_for(ns), kGThreads, 0, st>>>(in.src_xyz, svals, ns, 3, sx);
    if (!chk()) return e;
    g_gather<<<grid_for(ns), kGThreads, 0, st>>>(in.density, svals, ns, 3, sd);
    if (!chk()) return e;
    g_gather<<<grid_for(ns), kGThreads, 0, st>>>(in.weight, svals, ns, 1, sw);
    if (!chk()) return e;
    if (in.kernel) {
        g_gather<<<grid_for(ns), kGThreads, 0, st>>>(in.normal, svals, ns, 3, sn);
        if (!chk()) return e;
    }
    g_gather<<<grid_for(nt), kGThreads, 0, st>>>(in.trg_xyz, tvals, nt, 3, tx);
    if (!chk()) return e;

    SumInputs p{};
    p.kernel = in.kernel;
    p.mixed = 0;                               // the correction is always float64
    p.n_src = ns;
    p.n_trg = nt;
    p.src_xyz = sx;
    p.density = sd;
    p.weight = sw;
    p.normal = in.kernel ? sn : nullptr;
    p.trg_xyz = tx;
    p.excl = 0;
    p.pref = in.pref;
    const KernelTimer none{};
    if ((e = launch_p2p_csr(p, ng, sofs, tofs, uofs, ul, ng, u, 0, base + l.off_p2p, st, none)) != hipSuccess)
        return e;
    g_subtract<<<grid_for(nt), kGThreads, 0, st>>>(u, tvals, nt, status, out);
    chk();
    return e;
}

}  // namespace stokes
