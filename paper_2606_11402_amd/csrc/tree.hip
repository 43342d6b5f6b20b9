// The bit-reversed left-balanced k-d tree of Sec. 2.2 built on the device by
// sorts, one tree level at a time (Sec. 2.3, last paragraph: the tree on the
// GPU from sort passes).
//
// The tree is the one graph_build makes on the host: the node of slot t
// covers a set S of points; its split dimension is the one of widest extent
// of S (max - min in double, the lowest dimension on ties); its point is the
// one of rank |S|/2 in S by the key (coordinate in that dimension, input
// index), -0.0 and +0.0 counting as equal coordinates; the points ranked
// below go to the left child (slot t + 2^level(t)), those above to the right
// child (slot t + 2^(level(t)+1)).  Every node depends only on its set, so
// any procedure that reproduces the sets reproduces the tree bit for bit.
//
// Level L holds the segments j = slot - (2^L - 1), j < 2^L.  Per level:
//   1. the split dimension of every segment from its min / max per
//      dimension (gathered at the end of the previous level);
//   2. a stable radix sort of all points, in input order, by the ordered
//      bits of their coordinate in their segment's dimension, then a stable
//      radix sort by segment (finished points last): every segment becomes
//      a contiguous run ordered by (coordinate, input index);
//   3. the point of rank |S|/2 of each run is the node's point; the runs
//      below and above it are the children's sets, already contiguous, so
//      their min / max come from a segmented reduction over each wave and
//      one atomic per run and dimension (integer min / max on order-
//      preserving bits: the result does not depend on the order).
// The sizes of all segments follow from N alone (left-balanced).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>

#include "status.h"
#include "vecchia.h"

namespace {

constexpr int kTreeBlock = 256;

// Order-preserving bits of a double (NaN excluded by the caller), with -0.0
// mapped to +0.0 so that the two zeros compare equal as in the host build.
__device__ __forceinline__ uint64_t ordered_bits(double v) {
    if (v == 0.0) v = 0.0;
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double from_ordered(uint64_t o) {
    const uint64_t u = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double((long long)u);
}

struct TreeScratch {
    uint64_t *key_a, *key_b;        // N: coordinate keys
    uint32_t *seg_a, *seg_b;        // N: segment keys
    int32_t *id_a, *id_b, *id_c;    // N: input indices
    int32_t* seg_of;                // N: segment of each input point at this level, -1 once placed
    int32_t *size_cur, *size_nxt;   // max segments: sizes of this / the next level's segments
    int32_t* start;                 // max segments: first position of each run
    int32_t* dim;                   // max segments: split dimension
    uint64_t *mm_cur, *mm_nxt;      // max segments x 6: min (3) then max (3), ordered bits
    void* cub;                      // radix sort / scan temporary storage
    size_t cub_bytes;
};

int64_t max_segments(int64_t n) {
    int64_t s = 1;
    while (s * 2 <= n) s *= 2;       // 2^floor(log2 n): the deepest level's width
    return s;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

size_t cub_bytes_for(int64_t n, int64_t segs) {
    size_t a = 0, b = 0, c = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, a, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                       (int32_t*)nullptr, (int)n);
    hipcub::DeviceRadixSort::SortPairs(nullptr, b, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                       (int32_t*)nullptr, (int)n);
    hipcub::DeviceScan::ExclusiveSum(nullptr, c, (int32_t*)nullptr, (int32_t*)nullptr, (int)segs);
    return std::max(a, std::max(b, c));
}

// Carve the scratch buffer; returns the bytes needed (base may be null).
size_t carve(char* base, int64_t n, TreeScratch* s) {
    const int64_t segs = max_segments(n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    s->key_a = (uint64_t*)take(8 * (size_t)n);
    s->key_b = (uint64_t*)take(8 * (size_t)n);
    s->seg_a = (uint32_t*)take(4 * (size_t)n);
    s->seg_b = (uint32_t*)take(4 * (size_t)n);
    s->id_a = (int32_t*)take(4 * (size_t)n);
    s->id_b = (int32_t*)take(4 * (size_t)n);
    s->id_c = (int32_t*)take(4 * (size_t)n);
    s->seg_of = (int32_t*)take(4 * (size_t)n);
    s->size_cur = (int32_t*)take(4 * (size_t)segs);
    s->size_nxt = (int32_t*)take(4 * (size_t)segs);
    s->start = (int32_t*)take(4 * (size_t)segs);
    s->dim = (int32_t*)take(4 * (size_t)segs);
    s->mm_cur = (uint64_t*)take(48 * (size_t)segs);
    s->mm_nxt = (uint64_t*)take(48 * (size_t)segs);
    s->cub_bytes = cub_bytes_for(n, segs);
    s->cub = take(s->cub_bytes);
    return off;
}

__global__ __launch_bounds__(kTreeBlock) void init_kernel(int32_t* __restrict__ seg_of, int32_t* __restrict__ size,
                                                          uint64_t* __restrict__ mm, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    if (i < n) seg_of[i] = 0;
    if (i == 0) size[0] = (int32_t)n;
    if (i < 3) {
        mm[i] = ~0ull;          // min: start at the largest key
        mm[3 + i] = 0ull;       // max: start at the smallest
    }
}

// Reset the next level's min / max slots of the segments [0, segs).
__global__ __launch_bounds__(kTreeBlock) void mm_reset_kernel(uint64_t* __restrict__ mm, int64_t segs) {
    const int64_t j = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    if (j >= segs) return;
    for (int c = 0; c < 3; ++c) {
        mm[6 * j + c] = ~0ull;
        mm[6 * j + 3 + c] = 0ull;
    }
}

// Min / max of the points of consecutive positions grouped by run label
// (label < 0: no run): a segmented reduction over each wave, then one atomic
// per run, dimension and bound from the last lane of the run.
__device__ __forceinline__ void run_minmax(int label, const uint64_t* v, uint64_t* mm) {
    const int lane = threadIdx.x & 63;
    uint64_t lo[3] = {v[0], v[1], v[2]}, hi[3] = {v[0], v[1], v[2]};
    for (int off = 1; off < 64; off <<= 1) {
        const int other = __shfl_up(label, off, 64);
        uint64_t olo[3], ohi[3];
        for (int c = 0; c < 3; ++c) {
            olo[c] = __shfl_up(lo[c], off, 64);
            ohi[c] = __shfl_up(hi[c], off, 64);
        }
        if (lane >= off && other == label) {
            for (int c = 0; c < 3; ++c) {
                lo[c] = olo[c] < lo[c] ? olo[c] : lo[c];
                hi[c] = ohi[c] > hi[c] ? ohi[c] : hi[c];
            }
        }
    }
    const int next = __shfl_down(label, 1, 64);
    const bool last = lane == 63 || next != label;
    if (label >= 0 && last) {
        for (int c = 0; c < 3; ++c) {
            atomicMin((unsigned long long*)&mm[6 * (int64_t)label + c], (unsigned long long)lo[c]);
            atomicMax((unsigned long long*)&mm[6 * (int64_t)label + 3 + c], (unsigned long long)hi[c]);
        }
    }
}

// Level 0: min / max over all points (one run).
__global__ __launch_bounds__(kTreeBlock) void root_minmax_kernel(const double* __restrict__ x, int64_t n,
                                                                 uint64_t* __restrict__ mm) {
    const int64_t i = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    uint64_t v[3] = {0, 0, 0};
    int label = -1;
    if (i < n) {
        label = 0;
        for (int c = 0; c < 3; ++c) v[c] = ordered_bits(x[3 * i + c]);
    }
    run_minmax(label, v, mm);
}

// Split dimension of every segment: widest max - min over the first d
// dimensions, the lowest on ties (as the host's widest_dim).
__global__ __launch_bounds__(kTreeBlock) void dim_kernel(const uint64_t* __restrict__ mm, const int32_t* __restrict__ size,
                                                         int32_t* __restrict__ dim, int64_t segs, int d) {
    const int64_t j = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    if (j >= segs || size[j] <= 0) return;
    int best = 0;
    double bext = from_ordered(mm[6 * j + 3]) - from_ordered(mm[6 * j]);
    for (int c = 1; c < d; ++c) {
        const double e = from_ordered(mm[6 * j + 3 + c]) - from_ordered(mm[6 * j + c]);
        if (e > bext) {
            bext = e;
            best = c;
        }
    }
    dim[j] = best;
}

// Keys in input order: the coordinate in the segment's dimension.
__global__ __launch_bounds__(kTreeBlock) void key_kernel(const double* __restrict__ x, const int32_t* __restrict__ seg_of,
                                                         const int32_t* __restrict__ dim, int64_t n,
                                                         uint64_t* __restrict__ key, int32_t* __restrict__ id) {
    const int64_t i = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t j = seg_of[i];
    key[i] = j >= 0 ? ordered_bits(x[3 * i + dim[j]]) : 0ull;
    id[i] = (int32_t)i;
}

// Segment keys in the coordinate order; placed points get `done`, which
// sorts after every segment.
__global__ __launch_bounds__(kTreeBlock) void segkey_kernel(const int32_t* __restrict__ seg_of,
                                                            const int32_t* __restrict__ id, int64_t n, uint32_t done,
                                                            uint32_t* __restrict__ segk) {
    const int64_t p = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    if (p >= n) return;
    const int32_t j = seg_of[id[p]];
    segk[p] = j >= 0 ? (uint32_t)j : done;
}

// Place the node points of level L and hand every other point of a run to
// its child; gather the children's min / max.
__global__ __launch_bounds__(kTreeBlock) void assign_kernel(const double* __restrict__ x, const uint32_t* __restrict__ segk,
                                                            const int32_t* __restrict__ id, int64_t active,
                                                            const int32_t* __restrict__ start,
                                                            const int32_t* __restrict__ size,
                                                            const int32_t* __restrict__ dim, int64_t level_first,
                                                            int64_t segs, int64_t next_cap, int32_t* __restrict__ seg_of,
                                                            int32_t* __restrict__ tree_perm, int32_t* __restrict__ sdim,
                                                            uint64_t* __restrict__ mm_next) {
    const int64_t p = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    int label = -1;
    uint64_t v[3] = {0, 0, 0};
    if (p < active) {
        const int64_t j = segk[p];
        const int32_t i = id[p];
        const int64_t r = p - start[j];
        const int64_t m = size[j] / 2;
        if (r == m) {
            tree_perm[level_first + j] = i;
            sdim[level_first + j] = dim[j];
            seg_of[i] = -1;
        } else if (r >= 0 && r < size[j]) {
            // a child exists only above the deepest level, where every
            // segment holds at most its node point; next_cap bounds it anyway
            const int64_t child = r < m ? j : j + segs;
            if (child < next_cap) {
                seg_of[i] = (int32_t)child;
                label = (int)child;
                for (int c = 0; c < 3; ++c) v[c] = ordered_bits(x[3 * (int64_t)i + c]);
            }
        }
    }
    run_minmax(label, v, mm_next);
}

// Sizes of the next level: left child j gets m, right child j + segs the rest.
__global__ __launch_bounds__(kTreeBlock) void child_size_kernel(const int32_t* __restrict__ size,
                                                                int32_t* __restrict__ next, int64_t segs) {
    const int64_t j = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    if (j >= segs) return;
    const int32_t s = size[j];
    const int32_t m = s / 2;
    next[j] = s > 0 ? m : 0;
    next[j + segs] = s > 0 ? s - m - 1 : 0;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kTreeBlock - 1) / kTreeBlock); }

}  // namespace

extern "C" int graph_tree_scratch_bytes(int64_t n, size_t* bytes) {
    vecchia_clear_error();
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "graph_tree_scratch_bytes: bytes is NULL");
    if (n < 1 || n >= (int64_t(1) << 31))
        return vecchia_set_error(VECCHIA_EINVAL, "graph_tree_scratch_bytes: need 1 <= N < 2^31");
    TreeScratch s;
    *bytes = carve(nullptr, n, &s);
    return VECCHIA_OK;
}

extern "C" int graph_tree_device(const double* x, int64_t n, int32_t d, int32_t* tree_perm, int32_t* sdim,
                                 void* scratch, size_t scratch_bytes, void* stream) {
    vecchia_clear_error();
    if (!x || !tree_perm || !sdim || !scratch)
        return vecchia_set_error(VECCHIA_EINVAL, "graph_tree_device: NULL argument");
    if (n < 1 || n >= (int64_t(1) << 31) || d < 1 || d > 3)
        return vecchia_set_error(VECCHIA_EINVAL, "graph_tree_device: need 1 <= N < 2^31 and 1 <= d <= 3");
    if (reinterpret_cast<uintptr_t>(scratch) & 255)
        return vecchia_set_error(VECCHIA_EINVAL, "graph_tree_device: scratch must be 256-byte aligned");
    TreeScratch s;
    const size_t need = carve(static_cast<char*>(scratch), n, &s);
    if (scratch_bytes < need)
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_tree_device: scratch has %zu bytes, needs %zu", scratch_bytes,
                                 need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    auto check = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
        return e == hipSuccess;
    };
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(n)), dim3(kTreeBlock), 0, st, s.seg_of, s.size_cur, s.mm_cur, n);
    hipLaunchKernelGGL(root_minmax_kernel, dim3(blocks_for(n)), dim3(kTreeBlock), 0, st, x, n, s.mm_cur);
    check(hipGetLastError());
    const int64_t max_segs = max_segments(n);
    int64_t placed = 0;
    for (int level = 0; e == hipSuccess && placed < n; ++level) {
        const int64_t segs = int64_t(1) << level;         // segments of this level (some may be empty)
        if (segs > max_segs) {
            e = hipErrorInvalidValue;                       // cannot happen for a left-balanced tree
            break;
        }
        const int64_t active = n - placed;                  // points not yet placed
        hipLaunchKernelGGL(dim_kernel, dim3(blocks_for(segs)), dim3(kTreeBlock), 0, st, s.mm_cur, s.size_cur, s.dim,
                           segs, d);
        hipLaunchKernelGGL(key_kernel, dim3(blocks_for(n)), dim3(kTreeBlock), 0, st, x, s.seg_of, s.dim, n, s.key_a,
                           s.id_a);
        size_t cb = s.cub_bytes;
        if (!check(hipGetLastError())) break;
        if (!check(hipcub::DeviceRadixSort::SortPairs(s.cub, cb, s.key_a, s.key_b, s.id_a, s.id_b, (int)n, 0, 64, st)))
            break;
        hipLaunchKernelGGL(segkey_kernel, dim3(blocks_for(n)), dim3(kTreeBlock), 0, st, s.seg_of, s.id_b, n,
                           (uint32_t)segs, s.seg_a);
        if (!check(hipGetLastError())) break;
        int bits = 1;
        while ((int64_t(1) << bits) <= segs) ++bits;       // segment keys and `done` = segs fit in `bits` bits
        cb = s.cub_bytes;
        if (!check(hipcub::DeviceRadixSort::SortPairs(s.cub, cb, s.seg_a, s.seg_b, s.id_b, s.id_c, (int)n, 0, bits,
                                                      st)))
            break;
        cb = s.cub_bytes;
        if (!check(hipcub::DeviceScan::ExclusiveSum(s.cub, cb, s.size_cur, s.start, (int)segs, st))) break;
        const int64_t next_segs = std::min<int64_t>(2 * segs, max_segs);
        hipLaunchKernelGGL(mm_reset_kernel, dim3(blocks_for(next_segs)), dim3(kTreeBlock), 0, st, s.mm_nxt, next_segs);
        hipLaunchKernelGGL(assign_kernel, dim3(blocks_for(active)), dim3(kTreeBlock), 0, st, x, s.seg_b, s.id_c, active,
                           s.start, s.size_cur, s.dim, segs - 1, segs, max_segs, s.seg_of, tree_perm, sdim,
                           s.mm_nxt);
        if (2 * segs <= max_segs)
            hipLaunchKernelGGL(child_size_kernel, dim3(blocks_for(segs)), dim3(kTreeBlock), 0, st, s.size_cur,
                               s.size_nxt, segs);
        if (!check(hipGetLastError())) break;
        // the segment sizes of one level differ by at most one, so every
        // level but the last is full: level L places min(2^L, N - (2^L - 1))
        placed += std::min<int64_t>(segs, n - (segs - 1));
        std::swap(s.size_cur, s.size_nxt);
        std::swap(s.mm_cur, s.mm_nxt);
    }
    if (e != hipSuccess) return vecchia_set_error(VECCHIA_EHIP, "graph_tree_device: %s", hipGetErrorString(e));
    return VECCHIA_OK;
}
