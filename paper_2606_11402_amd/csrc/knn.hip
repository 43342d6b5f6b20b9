// Preceding k-NN query on the device (Sec. 2.1; the GPU search of Sec. 2.3's
// last paragraph): for every slot i >= n0, the k slots j < i with the
// smallest key (D, j), D = ((dx*dx + dy*dy) + dz*dz) in double without
// contraction.  One thread per query walks the query tree restricted to the
// prefix {0 .. i-1} (every parent precedes its children, so the prefix is a
// k-d tree itself), near side first.  The candidates are kept sorted by key
// in registers (an unrolled insertion network over KP entries); a far
// subtree is skipped only when its plane bound is strictly greater than the
// current k-th best key's D, which is exact under monotone rounding, so the
// result equals the brute-force search bit for bit (the host builder's
// search makes the same decisions).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "knn.h"
#include "lanes.h"
#include "status.h"
#include "vecchia.h"

#pragma clang fp contract(off)

namespace {

__device__ __forceinline__ int tree_level_d(int64_t t) { return 63 - __clzll((unsigned long long)(t + 1)); }

__device__ __forceinline__ bool key_less(double da, int32_t sa, double db, int32_t sb) {
    return da < db || (da == db && sa < sb);
}

// A depth-first walk keeps at most one pending far subtree per tree level
// plus the near child, so a tree of fewer than 2^31 points (31 levels) never
// holds more than 32 entries; the bound checks below only keep memory safe.
constexpr int kKnnStack = 64;

template <int KP>
__global__ __launch_bounds__(256) void knn_kernel(const KnnNode* __restrict__ nodes, const int32_t* __restrict__ rank_of,
                                                  int64_t n, int k, int n0, int32_t* __restrict__ rows) {
    const int64_t i = (int64_t)n0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const KnnNode qn = nodes[rank_of[i]];
    const double q0 = qn.c[0], q1 = qn.c[1], q2 = qn.c[2];
    const int cap = (int)(i < k ? i : k);
    double dist[KP];
    int32_t sl[KP];
    static_for<0, KP>([&](auto MI) {
        dist[(int)MI] = INFINITY;
        sl[(int)MI] = 0x7fffffff;
    });
    int size = 0;
    double wd = INFINITY;                 // key of the k-th best once full
    int32_t ws = 0x7fffffff;
    int32_t st_rank[kKnnStack];
    double st_bound[kKnnStack];
    int sp = 0;
    st_rank[sp] = rank_of[0];
    st_bound[sp] = 0.0;
    ++sp;
    while (sp > 0) {
        --sp;
        const int32_t rank = st_rank[sp];
        const double bound = st_bound[sp];
        if (size == cap && bound > wd) continue;
        const KnnNode nd = nodes[rank];
        const int64_t t = nd.slot;
        const double dx = q0 - nd.c[0], dy = q1 - nd.c[1], dz = q2 - nd.c[2];
        const double dd = (dx * dx + dy * dy) + dz * dz;
        if (size < cap || key_less(dd, (int32_t)t, wd, ws)) {
            // sorted insertion of (dd, t); entries past cap fall off the end
            static_for<0, KP>([&](auto MJ) {
                constexpr int m = KP - 1 - (int)MJ;
                if constexpr (m > 0) {
                    const bool prev = key_less(dd, (int32_t)t, dist[m - 1], sl[m - 1]);
                    const bool here = !prev && key_less(dd, (int32_t)t, dist[m], sl[m]);
                    dist[m] = prev ? dist[m - 1] : (here ? dd : dist[m]);
                    sl[m] = prev ? sl[m - 1] : (here ? (int32_t)t : sl[m]);
                } else {
                    const bool here = key_less(dd, (int32_t)t, dist[0], sl[0]);
                    dist[0] = here ? dd : dist[0];
                    sl[0] = here ? (int32_t)t : sl[0];
                }
            });
            size = size < cap ? size + 1 : cap;
            if (size == cap) {
                static_for<0, KP>([&](auto MI) {
                    constexpr int m = MI;
                    if (m == cap - 1) {
                        wd = dist[m];
                        ws = sl[m];
                    }
                });
            }
        }
        const int s = nd.sdim;
        const double diff = (s == 0 ? q0 : (s == 1 ? q1 : q2)) - (s == 0 ? nd.c[0] : (s == 1 ? nd.c[1] : nd.c[2]));
        const int lvl = tree_level_d(t);
        const int64_t l = t + (int64_t(1) << lvl), r = t + (int64_t(2) << lvl);
        const bool left_near = diff < 0.0;
        const int64_t near_c = left_near ? l : r, far_c = left_near ? r : l;
        const int32_t near_r = left_near ? nd.left : nd.right, far_r = left_near ? nd.right : nd.left;
        const double plane = fmax(bound, diff * diff);
        if (far_c < i && !(size == cap && plane > wd) && sp < kKnnStack) {
            st_rank[sp] = far_r;
            st_bound[sp] = plane;
            ++sp;
        }
        if (near_c < i && sp < kKnnStack) {
            st_rank[sp] = near_r;
            st_bound[sp] = bound;
            ++sp;
        }
    }
    int32_t* out = rows + (i - n0) * (int64_t)k;
    static_for<0, KP>([&](auto MI) {
        constexpr int m = MI;
        if (m < k) out[m] = m < cap ? sl[m] : -1;
    });
}

}  // namespace

extern "C" int graph_knn_device(const void* nodes, const int32_t* rank_of, int64_t n, int32_t d, int32_t k, int32_t n0,
                                int32_t* rows, void* stream) {
    vecchia_clear_error();
    if (!nodes || !rank_of || !rows) return vecchia_set_error(VECCHIA_EINVAL, "graph_knn_device: NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31) || d < 1 || d > 3 || n0 < 1 || n0 > n)
        return vecchia_set_error(VECCHIA_EINVAL, "graph_knn_device: need 1 <= n0 <= N < 2^31 and 1 <= d <= 3");
    if (k < 1) return vecchia_set_error(VECCHIA_EINVAL, "graph_knn_device: need k >= 1");
    if (k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "graph_knn_device: k=%d exceeds the compiled maximum %d", k,
                                 VECCHIA_KMAX);
    const int64_t q = n - n0;
    if (q == 0) return VECCHIA_OK;
    const dim3 grid((unsigned)((q + 255) / 256)), block(256);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const KnnNode* nd = static_cast<const KnnNode*>(nodes);
    const int kp = vecchia_padded_k(k);
    switch (kp) {
        case 8: hipLaunchKernelGGL((knn_kernel<8>), grid, block, 0, s, nd, rank_of, n, k, n0, rows); break;
        case 16: hipLaunchKernelGGL((knn_kernel<16>), grid, block, 0, s, nd, rank_of, n, k, n0, rows); break;
        case 32: hipLaunchKernelGGL((knn_kernel<32>), grid, block, 0, s, nd, rank_of, n, k, n0, rows); break;
        default: hipLaunchKernelGGL((knn_kernel<64>), grid, block, 0, s, nd, rank_of, n, k, n0, rows); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return vecchia_set_error(VECCHIA_EHIP, "graph_knn_device: %s", hipGetErrorString(e));
    return VECCHIA_OK;
}

// ---- depths (Sec. 2.2: d_i = 1 + max over the neighbours' depths, the
// dense block at depth 0) as the parallel fixpoint of that recurrence: every
// sparse slot starts at 1 and each sweep raises d_i to 1 + max d_j, in place.
// Depths only grow and are bounded by the longest chain of the neighbour
// graph, so the sweeps end; the fixpoint is the longest-path depth, which is
// unique, so neither the order of the updates nor stale reads of a slot that
// another thread is raising change the result, only the number of sweeps.
// Sweeps over all slots at once advance a chain of neighbours by about one
// link each (measured: ~490 sweeps at 2^26); since every neighbour precedes
// its point, the slots are instead taken in consecutive blocks, in order:
// the depths of earlier blocks are final when a block starts, so a block
// needs only as many sweeps as the chains inside it are long, usually one
// or two.
namespace {

__global__ __launch_bounds__(256) void depth_init_kernel(int32_t* __restrict__ depth, int64_t n, int n0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) depth[i] = i < n0 ? 0 : 1;
}

__global__ __launch_bounds__(256) void depth_sweep_kernel(const int32_t* __restrict__ rows, int64_t lo, int64_t hi,
                                                          int k, int n0, int32_t* depth,
                                                          int32_t* __restrict__ changed) {
    const int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hi) return;
    const int32_t* row = rows + (i - n0) * (int64_t)k;
    int32_t m = 0;
    for (int q = 0; q < k; ++q) {
        const int32_t j = row[q];
        if (j < 0) break;                         // padding only at the end of a row
        m = max(m, __atomic_load_n(depth + j, __ATOMIC_RELAXED));
    }
    if (m + 1 > depth[i]) {
        __atomic_store_n(depth + i, m + 1, __ATOMIC_RELAXED);
        *changed = 1;
    }
}

__global__ void flag_zero_kernel(int32_t* __restrict__ flag) { *flag = 0; }

}  // namespace

extern "C" int graph_depth_device(const int32_t* rows, int64_t n, int32_t k, int32_t n0, int32_t* depth,
                                  int32_t* scratch, void* stream, int32_t* sweeps) {
    vecchia_clear_error();
    if (!rows || !depth || !scratch) return vecchia_set_error(VECCHIA_EINVAL, "graph_depth_device: NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31) || n0 < 1 || n0 > n || k < 1)
        return vecchia_set_error(VECCHIA_EINVAL, "graph_depth_device: need 1 <= n0 <= N < 2^31 and k >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(depth_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, depth, n, n0);
    hipError_t e = hipGetLastError();
    int32_t done_sweeps = 0;
    // per block: sweeps until one changes nothing (at most one per slot of the
    // block, the longest chain inside it); the test costs a synchronisation,
    // so it follows every second sweep (an extra sweep after the fixpoint
    // changes nothing)
    constexpr int64_t kDepthBlock = int64_t(1) << 16;
    constexpr int kSweepsPerTest = 2;
    for (int64_t lo = n0; e == hipSuccess && lo < n; lo += kDepthBlock) {
        const int64_t hi = std::min(n, lo + kDepthBlock);
        for (int64_t round = 0; round * kSweepsPerTest <= hi - lo; ++round) {
            hipLaunchKernelGGL(flag_zero_kernel, dim3(1), dim3(1), 0, s, scratch);
            for (int t = 0; t < kSweepsPerTest; ++t)
                hipLaunchKernelGGL(depth_sweep_kernel, dim3((unsigned)((hi - lo + 255) / 256)), dim3(256), 0, s, rows,
                                   lo, hi, k, n0, depth, scratch);
            done_sweeps += kSweepsPerTest;
            int32_t changed = 1;
            if ((e = hipGetLastError()) != hipSuccess) break;
            if ((e = hipMemcpyAsync(&changed, scratch, sizeof(changed), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
            if (!changed) break;
        }
    }
    if (e != hipSuccess) return vecchia_set_error(VECCHIA_EHIP, "graph_depth_device: %s", hipGetErrorString(e));
    if (sweeps) *sweeps = done_sweeps;
    return VECCHIA_OK;
}
