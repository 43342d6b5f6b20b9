// Host graph build of the Vecchia hot path: bit-reversed k-d tree order,
// k nearest preceding neighbours, depth batches and storage order.
//
// Sec. 2.2 ("Tree ordering", "Bit-reversed ordering"): the slot t at tree
// level l = floor(log2(t+1)) has children t + 2^l (left) and t + 2^(l+1)
// (right); with this layout every level but the last is full, the last one is
// filled in bit-reversed position order, and each node's left subtree holds
// floor(n/2) of the n points under it.  A node therefore keeps the point of
// rank floor(n/2) along its split dimension; the split dimension is the one
// of widest extent (lowest index on ties) and ranks are taken on the key
// (coordinate, input index).
//
// Sec. 2.1: c(i) = the k nearest points among the slots j < i, key (D, j)
// with D = ((dx*dx + dy*dy) + dz*dz) in double and no contraction (this file
// is compiled with -ffp-contract=off).  Because every parent precedes its
// children, the slots {0..i-1} form a k-d tree themselves and the query walks
// only that prefix.  A far subtree is skipped only when the squared distance
// to its splitting plane is strictly greater than the current k-th best D:
// that plane distance, rounded, is a lower bound of the rounded D of every
// point behind the plane, so ties are never lost and the result equals the
// brute-force search bit for bit.
//
// Sec. 2.2 ("Batch construction"): d_i = 1 + max_{j in c(i)} d_j in slot
// order; the dense block (slots < n0) has depth 0.  Storage order: the dense
// block in slot order, then the batches in increasing depth; inside a batch
// the points follow the in-order sequence of the tree, which keeps spatial
// neighbours close in memory for the gathers on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "graph_internal.h"
#include "knn.h"
#include "status.h"
#include "vecchia.h"

namespace {

inline int tree_level(int64_t t) { return 63 - __builtin_clzll((uint64_t)(t + 1)); }
inline int64_t left_child(int64_t t) { return t + (int64_t(1) << tree_level(t)); }
inline int64_t right_child(int64_t t) { return t + (int64_t(2) << tree_level(t)); }

template <class F>
void parallel_for(int64_t n, int64_t grain, int nthreads, F&& f) {
    if (n <= 0) return;
    if (nthreads <= 1 || n <= grain) {
        f(int64_t(0), n);
        return;
    }
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        for (;;) {
            int64_t a = next.fetch_add(grain);
            if (a >= n) break;
            f(a, std::min(n, a + grain));
        }
    };
    int nt = (int)std::min<int64_t>(nthreads, (n + grain - 1) / grain);
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
}

struct TreePoint {
    double c[3];
    int32_t id;
    int32_t pad;
};

struct Task {
    int64_t slot, lo, hi;
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Split dimension of pts[lo, hi): widest extent, lowest index on ties.
int widest_dim(const TreePoint* pts, int64_t lo, int64_t hi, int d, int nthreads) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t big = int64_t(1) << 22;
    if (hi - lo >= big && nthreads > 1) {
        int64_t chunks = (hi - lo + big - 1) / big;
        std::vector<double> pmn(chunks * 3, INFINITY), pmx(chunks * 3, -INFINITY);
        parallel_for(chunks, 1, nthreads, [&](int64_t a, int64_t b) {
            for (int64_t ch = a; ch < b; ++ch) {
                int64_t s = lo + ch * big, e = std::min(hi, s + big);
                for (int64_t p = s; p < e; ++p)
                    for (int c = 0; c < d; ++c) {
                        pmn[ch * 3 + c] = std::min(pmn[ch * 3 + c], pts[p].c[c]);
                        pmx[ch * 3 + c] = std::max(pmx[ch * 3 + c], pts[p].c[c]);
                    }
            }
        });
        for (int64_t ch = 0; ch < chunks; ++ch)
            for (int c = 0; c < d; ++c) {
                mn[c] = std::min(mn[c], pmn[ch * 3 + c]);
                mx[c] = std::max(mx[c], pmx[ch * 3 + c]);
            }
    } else {
        for (int64_t p = lo; p < hi; ++p)
            for (int c = 0; c < d; ++c) {
                mn[c] = std::min(mn[c], pts[p].c[c]);
                mx[c] = std::max(mx[c], pts[p].c[c]);
            }
    }
    int best = 0;
    double bext = mx[0] - mn[0];
    for (int c = 1; c < d; ++c) {
        double e = mx[c] - mn[c];
        if (e > bext) {
            bext = e;
            best = c;
        }
    }
    return best;
}

void build_tree(vecchia_graph& g, const double* x, int nthreads) {
    const int64_t n = g.n;
    const int d = g.d;
    std::vector<TreePoint> pts(n);
    parallel_for(n, 1 << 16, nthreads, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            for (int c = 0; c < 3; ++c) pts[i].c[c] = c < d ? x[i * d + c] : 0.0;
            pts[i].id = (int32_t)i;
            pts[i].pad = 0;
        }
    });
    g.tree_perm.assign(n, -1);
    g.sdim.assign(n, 0);
    std::vector<Task> cur{{0, 0, n}}, nxt;
    while (!cur.empty()) {
        nxt.assign(cur.size() * 2, Task{-1, 0, 0});
        // few large tasks: give each the whole pool for its extent scan
        int inner = cur.size() < (size_t)nthreads ? std::max(1, nthreads / (int)cur.size()) : 1;
        parallel_for((int64_t)cur.size(), 1, nthreads, [&](int64_t a, int64_t b) {
            for (int64_t ti = a; ti < b; ++ti) {
                const Task tk = cur[ti];
                const int64_t cnt = tk.hi - tk.lo;
                const int s = widest_dim(pts.data(), tk.lo, tk.hi, d, inner);
                const int64_t m = cnt / 2;
                std::nth_element(pts.begin() + tk.lo, pts.begin() + tk.lo + m, pts.begin() + tk.hi,
                                 [s](const TreePoint& p, const TreePoint& q) {
                                     return p.c[s] < q.c[s] || (p.c[s] == q.c[s] && p.id < q.id);
                                 });
                g.tree_perm[tk.slot] = pts[tk.lo + m].id;
                g.sdim[tk.slot] = (int8_t)s;
                if (m > 0) nxt[2 * ti] = Task{left_child(tk.slot), tk.lo, tk.lo + m};
                if (cnt - m - 1 > 0) nxt[2 * ti + 1] = Task{right_child(tk.slot), tk.lo + m + 1, tk.hi};
            }
        });
        cur.clear();
        for (const Task& t : nxt)
            if (t.slot >= 0) cur.push_back(t);
    }
    g.xs.resize(n * 3);
    parallel_for(n, 1 << 16, nthreads, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) {
            const int64_t i = g.tree_perm[t];
            for (int c = 0; c < 3; ++c) g.xs[t * 3 + c] = c < d ? x[i * d + c] : 0.0;
        }
    });
}

// Max-heap of the best candidates by (D, slot).
struct Candidates {
    double dist[VECCHIA_KMAX];
    int32_t slot[VECCHIA_KMAX];
    int size = 0, cap = 0;

    bool worse(int a, int b) const {  // entry a ranks after entry b
        return dist[a] > dist[b] || (dist[a] == dist[b] && slot[a] > slot[b]);
    }
    bool full() const { return size == cap; }
    double worst() const { return dist[0]; }
    void offer(double dd, int32_t s) {
        if (size < cap) {
            int i = size++;
            dist[i] = dd;
            slot[i] = s;
            while (i > 0) {
                int p = (i - 1) / 2;
                if (!worse(i, p)) break;
                std::swap(dist[i], dist[p]);
                std::swap(slot[i], slot[p]);
                i = p;
            }
            return;
        }
        if (dd > dist[0] || (dd == dist[0] && s > slot[0])) return;
        dist[0] = dd;
        slot[0] = s;
        int i = 0;
        for (;;) {
            int l = 2 * i + 1, r = l + 1, w = i;
            if (l < size && worse(l, w)) w = l;
            if (r < size && worse(r, w)) w = r;
            if (w == i) break;
            std::swap(dist[i], dist[w]);
            std::swap(slot[i], slot[w]);
            i = w;
        }
    }
};

inline double sqdist(const double* a, const double* b, int d) {
    double dx = a[0] - b[0];
    double acc = dx * dx;
    if (d > 1) {
        double dy = a[1] - b[1];
        acc = acc + dy * dy;
    }
    if (d > 2) {
        double dz = a[2] - b[2];
        acc = acc + dz * dz;
    }
    return acc;
}

// Query tree in in-order layout: the nodes of every subtree occupy one
// contiguous range of ranks, so the bottom of a search touches nearby memory.
struct QNode {
    double c[3];
    int32_t slot;
    int32_t left, right;   // in-order ranks of the children, -1 if absent
    int32_t sdim;
};

// In-order sequence of the tree.  The subtree sizes follow from N alone (a
// node's left subtree holds floor(m/2) of the m points under it, the right
// one the rest but the node), so the subtree of slot t covers the in-order
// ranks [lo_t, lo_t + m_t), the node itself has rank lo_t + floor(m_t/2),
// and the ranges of its children follow; one parallel pass per tree level,
// root first.
void inorder(vecchia_graph& g) {
    const int64_t n = g.n;
    g.seq.resize(n);
    g.rank_of.resize(n);
    std::vector<int32_t> lo(n), cnt(n);
    lo[0] = 0;
    cnt[0] = (int32_t)n;
    const int levels = tree_level(n - 1) + 1;
    for (int l = 0; l < levels; ++l) {
        const int64_t first = (int64_t(1) << l) - 1, last = std::min<int64_t>(n, (int64_t(2) << l) - 1);
        parallel_for(last - first, 1 << 15, g.nthreads, [&](int64_t a, int64_t b) {
            for (int64_t t = first + a; t < first + b; ++t) {
                const int64_t s = lo[t], m = cnt[t], h = m / 2;
                g.seq[s + h] = (int32_t)t;
                g.rank_of[t] = (int32_t)(s + h);
                const int64_t lc = left_child(t), rc = right_child(t);
                if (lc < n) {
                    lo[lc] = (int32_t)s;
                    cnt[lc] = (int32_t)h;
                }
                if (rc < n) {
                    lo[rc] = (int32_t)(s + h + 1);
                    cnt[rc] = (int32_t)(m - 1 - h);
                }
            }
        });
    }
}

// The k nearest slots j < i of slot i (Sec. 2.1), written ascending by
// (D, j) as in-order ranks.
void query_preceding(const vecchia_graph& g, const QNode* nodes, int64_t i, int32_t* out) {
    const double* q = &g.xs[i * 3];
    const int d = g.d;
    Candidates cand;
    cand.cap = (int)std::min<int64_t>(g.k, i);
    struct Item {
        int32_t rank;
        double bound;
    };
    Item stack[192];
    int sp = 0;
    stack[sp++] = Item{g.rank_of[0], 0.0};
    while (sp > 0) {
        const Item it = stack[--sp];
        if (cand.full() && it.bound > cand.worst()) continue;
        const QNode& nd = nodes[it.rank];
        const int64_t t = nd.slot;
        cand.offer(sqdist(q, nd.c, d), (int32_t)t);
        const int s = nd.sdim;
        const double diff = q[s] - nd.c[s];
        const int64_t l = left_child(t), r = right_child(t);
        const bool left_near = diff < 0.0;
        const int64_t near_c = left_near ? l : r, far_c = left_near ? r : l;
        const int32_t near_r = left_near ? nd.left : nd.right, far_r = left_near ? nd.right : nd.left;
        const double plane = std::max(it.bound, diff * diff);
        if (far_c < i && !(cand.full() && plane > cand.worst())) stack[sp++] = Item{far_r, plane};
        if (near_c < i) stack[sp++] = Item{near_r, it.bound};
    }
    const int m = cand.size;
    int32_t idx[VECCHIA_KMAX];
    for (int a = 0; a < m; ++a) idx[a] = a;
    std::sort(idx, idx + m, [&](int a, int b) {
        return cand.dist[a] < cand.dist[b] || (cand.dist[a] == cand.dist[b] && cand.slot[a] < cand.slot[b]);
    });
    for (int a = 0; a < m; ++a) out[a] = g.rank_of[cand.slot[idx[a]]];
    for (int a = m; a < g.k; ++a) out[a] = -1;
}

void build_neighbours(vecchia_graph& g, int nthreads) {
    const int64_t n = g.n, ns = g.n - g.n0;
    std::vector<QNode> nodes(n);
    parallel_for(n, 1 << 16, nthreads, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int64_t t = g.seq[r];
            QNode& nd = nodes[r];
            for (int c = 0; c < 3; ++c) nd.c[c] = g.xs[t * 3 + c];
            nd.slot = (int32_t)t;
            const int64_t l = left_child(t), rr = right_child(t);
            nd.left = l < n ? g.rank_of[l] : -1;
            nd.right = rr < n ? g.rank_of[rr] : -1;
            nd.sdim = g.sdim[t];
        }
    });
    g.nbr.resize((size_t)ns * g.k);
    // queries in in-order sequence: consecutive queries search the same region
    parallel_for(n, 2048, nthreads, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int64_t i = g.seq[r];
            if (i >= g.n0) query_preceding(g, nodes.data(), i, &g.nbr[(size_t)(i - g.n0) * g.k]);
        }
    });
}

// Depths in slot order (the recurrence of Sec. 2.2), kept in rank space so
// that the depths of a point's neighbours, its spatial neighbours, are read
// from nearby memory.  Slots are taken in blocks: the maximum over the
// neighbours in earlier blocks is taken in parallel (their depths are final),
// and only the rows that also have a neighbour inside the block (its depth
// still -1) are finished sequentially, in slot order.  Far into the order
// the neighbours of a point are spread over all preceding slots, so few rows
// need the sequential step.
void build_depth(vecchia_graph& g, int nthreads) {
    std::vector<int32_t> dr(g.n, 0);
    for (int64_t i = g.n0; i < g.n; ++i) dr[g.rank_of[i]] = -1;
    const int64_t block = 1 << 17;
    std::vector<int32_t> dm(block);
    std::vector<uint8_t> late(block);
    int32_t maxd = 0;
    for (int64_t a = g.n0; a < g.n; a += block) {
        const int64_t b = std::min(a + block, g.n);
        parallel_for(b - a, 2048, nthreads, [&](int64_t lo, int64_t hi) {
            for (int64_t i = a + lo; i < a + hi; ++i) {
                const int32_t* row = &g.nbr[(size_t)(i - g.n0) * g.k];
                int32_t m = 0;
                uint8_t l = 0;
                for (int q = 0; q < g.k; ++q) {
                    if (row[q] < 0) break;
                    const int32_t d = dr[row[q]];
                    l |= d < 0;
                    m = std::max(m, d);
                }
                dm[i - a] = m;
                late[i - a] = l;
            }
        });
        for (int64_t i = a; i < b; ++i) {
            int32_t m = dm[i - a];
            if (late[i - a]) {
                const int32_t* row = &g.nbr[(size_t)(i - g.n0) * g.k];
                for (int q = 0; q < g.k; ++q) {
                    if (row[q] < 0) break;
                    m = std::max(m, dr[row[q]]);
                }
            }
            dr[g.rank_of[i]] = m + 1;
            maxd = std::max(maxd, m + 1);
        }
    }
    g.depth.resize(g.n);
    for (int64_t t = 0; t < g.n; ++t) g.depth[t] = dr[g.rank_of[t]];
    g.n_levels = g.n > g.n0 ? maxd : 0;
}

void build_storage(vecchia_graph& g) {
    const int64_t n = g.n;
    const int L = g.n_levels;
    const int W = L + 2;
    // The sparse slots, taken in the in-order sequence, are sorted stably by
    // depth.  Counting sort over fixed chunks of the sequence: each chunk
    // counts its slots per depth, an exclusive prefix over (depth, chunk)
    // gives each chunk its first position in every batch, and the chunks then
    // place their slots independently -- the same order as one serial pass.
    const int nc = (int)std::max<int64_t>(1, std::min<int64_t>(g.nthreads, (n + (1 << 16) - 1) >> 16));
    const int64_t chunk = (n + nc - 1) / nc;
    std::vector<int64_t> cnt((size_t)nc * W, 0);
    parallel_for(nc, 1, nc, [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            int64_t* my = &cnt[(size_t)c * W];
            for (int64_t r = c * chunk; r < std::min(n, (c + 1) * chunk); ++r) {
                const int64_t t = g.seq[r];
                if (t >= g.n0) my[g.depth[t]]++;
            }
        }
    });
    g.level_ptr.assign(W, 0);
    g.level_ptr[1] = g.n0;
    for (int l = 1; l <= L; ++l) {
        int64_t off = g.level_ptr[l];
        for (int c = 0; c < nc; ++c) {
            const int64_t m = cnt[(size_t)c * W + l];
            cnt[(size_t)c * W + l] = off;
            off += m;
        }
        g.level_ptr[l + 1] = (int32_t)off;
    }
    g.order.assign(n, -1);
    g.pos.assign(n, -1);
    for (int64_t t = 0; t < g.n0; ++t) g.order[t] = (int32_t)t;
    // inside a batch: in-order sequence of the tree (spatially coherent)
    parallel_for(nc, 1, nc, [&](int64_t a, int64_t b) {
        for (int64_t c = a; c < b; ++c) {
            int64_t* fill = &cnt[(size_t)c * W];
            for (int64_t r = c * chunk; r < std::min(n, (c + 1) * chunk); ++r) {
                const int64_t t = g.seq[r];
                if (t >= g.n0) g.order[fill[g.depth[t]]++] = (int32_t)t;
            }
        }
    });
    parallel_for(n, 1 << 16, g.nthreads, [&](int64_t a, int64_t b) {
        for (int64_t s = a; s < b; ++s) g.pos[g.order[s]] = (int32_t)s;
    });
    g.pos_r.resize(n);
    parallel_for(n, 1 << 16, g.nthreads, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) g.pos_r[r] = g.pos[g.seq[r]];
    });
}

// Row of sparse point sp in the device order: storage positions ascending,
// padding (-1) last.  The points of a tile are spatial neighbours inside one
// batch, so with every row in this order the m-th gathers of a wave (of v in
// the forward and inverse, of coordinates in the factor) fall on nearly the
// same positions and touch few distinct cache lines; in distance order the
// m-th nearest neighbours of adjacent points are scattered.  The conditioning
// set, and with it every result up to rounding, does not depend on the order
// of its members (b is permuted alike).
void device_row(const vecchia_graph& g, int64_t sp, int32_t* out) {
    const int32_t t = g.order[g.n0 + sp];
    const int32_t* row = &g.nbr[(size_t)(t - g.n0) * g.k];
    for (int m = 0; m < g.k; ++m) out[m] = row[m] >= 0 ? g.pos_r[row[m]] : -1;
    std::sort(out, out + g.k, [](int32_t a, int32_t b) { return (uint32_t)a < (uint32_t)b; });
}

}  // namespace

namespace {

int check_build_args(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0, vecchia_graph** out,
                     const char* who) {
    if (!out) return vecchia_set_error(VECCHIA_EINVAL, "%s: out is NULL", who);
    *out = nullptr;
    if (!x) return vecchia_set_error(VECCHIA_EINVAL, "%s: x is NULL", who);
    if (n < 1 || n >= (int64_t(1) << 31)) return vecchia_set_error(VECCHIA_EINVAL, "%s: need 1 <= N < 2^31, got %lld", who, (long long)n);
    if (d < 1 || d > 3) return vecchia_set_error(VECCHIA_EINVAL, "%s: need 1 <= d <= 3, got %d", who, d);
    if (k < 1) return vecchia_set_error(VECCHIA_EINVAL, "%s: need k >= 1, got %d", who, k);
    if (k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "%s: k=%d exceeds the compiled maximum %d", who, k, VECCHIA_KMAX);
    if (n0 < 1 || n0 > n) return vecchia_set_error(VECCHIA_EINVAL, "%s: need 1 <= n0 <= N, got n0=%d", who, n0);
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(x[i])) return vecchia_set_error(VECCHIA_EINVAL, "%s: non-finite coordinate at point %lld", who, (long long)(i / d));
    return VECCHIA_OK;
}

// Tree order and in-order sequence (the part that the neighbour search,
// wherever it runs, needs first).
vecchia_graph* begin_graph(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0, int nthreads) {
    vecchia_graph* g = new vecchia_graph();
    g->n = n;
    g->d = d;
    g->k = k;
    g->kp = vecchia_padded_k(k);
    g->n0 = n0;
    g->nthreads = nthreads;
    auto t0 = std::chrono::steady_clock::now();
    build_tree(*g, x, nthreads);
    inorder(*g);
    g->times[0] = seconds_since(t0);
    return g;
}

double canon_zero(double v) { return v == 0.0 ? 0.0 : v; }

// Whether (perm, sdim) is the tree build_tree makes from x, checked without
// rebuilding it (Sec. 2.2): perm is a permutation; the split dimension of
// every slot is the widest extent of its subtree's points (the lowest on
// ties); every point of a slot's left subtree is below, every point of its
// right subtree above the slot's point by (coordinate in the split
// dimension, input index).  The subtree sizes are fixed by N (left-balanced
// slots), so these properties determine the tree.  One bottom-up pass
// (deepest level first) keeps, per subtree and dimension, the smallest and
// the largest (coordinate, index) key; a slot then compares its own key with
// the largest of its left subtree and the smallest of its right one.
// Returns the first failing slot, or -1.
int64_t check_tree(const double* x, int64_t n, int d, const int32_t* perm, const int32_t* sdim, int nthreads) {
    std::vector<uint8_t> seen(n, 0);
    for (int64_t t = 0; t < n; ++t) {
        const int32_t i = perm[t];
        if (i < 0 || i >= n || seen[i] || sdim[t] < 0 || sdim[t] >= d) return t;
        seen[i] = 1;
    }
    std::atomic<int64_t> bad(n);
    auto fail = [&](int64_t t) {
        int64_t cur = bad.load();
        while (t < cur && !bad.compare_exchange_weak(cur, t)) {
        }
    };
    struct Key {
        double c;
        int32_t id;
    };
    auto less = [](const Key& a, const Key& b) { return a.c < b.c || (a.c == b.c && a.id < b.id); };
    // not zeroed: an entry (slot, dimension < d) is written before any read of
    // it, since slots are visited deepest level first and read only their
    // children's entries
    std::unique_ptr<Key[]> lo(new Key[(size_t)n * 3]), hi(new Key[(size_t)n * 3]);
    const int levels = tree_level(n - 1) + 1;
    for (int l = levels - 1; l >= 0; --l) {
        const int64_t first = (int64_t(1) << l) - 1, last = std::min<int64_t>(n, (int64_t(2) << l) - 1);
        parallel_for(last - first, 1 << 12, nthreads, [&](int64_t a, int64_t b) {
            for (int64_t t = first + a; t < first + b; ++t) {
                const int32_t id = perm[t];
                const int s = sdim[t];
                const Key own{canon_zero(x[(int64_t)id * d + s]), id};
                const int64_t lc = left_child(t), rc = right_child(t);
                if (lc < n && !less(hi[lc * 3 + s], own)) fail(t);
                if (rc < n && !less(own, lo[rc * 3 + s])) fail(t);
                for (int c = 0; c < d; ++c) {
                    Key k{canon_zero(x[(int64_t)id * d + c]), id};
                    Key mn = k, mx = k;
                    for (int64_t ch : {lc, rc}) {
                        if (ch >= n) continue;
                        if (less(lo[ch * 3 + c], mn)) mn = lo[ch * 3 + c];
                        if (less(mx, hi[ch * 3 + c])) mx = hi[ch * 3 + c];
                    }
                    lo[t * 3 + c] = mn;
                    hi[t * 3 + c] = mx;
                }
                int best = 0;
                double bext = hi[t * 3].c - lo[t * 3].c;
                for (int c = 1; c < d; ++c) {
                    const double e = hi[t * 3 + c].c - lo[t * 3 + c].c;
                    if (e > bext) {
                        bext = e;
                        best = c;
                    }
                }
                if (s != best) fail(t);
            }
        });
        if (bad.load() < n) return bad.load();
    }
    return -1;
}

void finish_graph(vecchia_graph& g, const int32_t* depth = nullptr) {
    auto t0 = std::chrono::steady_clock::now();
    if (depth) {
        g.depth.assign(depth, depth + g.n);
        int32_t maxd = 0;
        for (int64_t t = g.n0; t < g.n; ++t) maxd = std::max(maxd, g.depth[t]);
        g.n_levels = g.n > g.n0 ? maxd : 0;
    } else {
        build_depth(g, g.nthreads);
    }
    g.times[2] = seconds_since(t0);
    t0 = std::chrono::steady_clock::now();
    build_storage(g);
    g.times[3] = seconds_since(t0);
    g.pending = false;
}

int threads_of(int32_t n_threads) {
    return n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
}

}  // namespace

extern "C" int graph_build(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0, int32_t n_threads,
                           vecchia_graph** out) {
    vecchia_clear_error();
    int rc = check_build_args(x, n, d, k, n0, out, "graph_build");
    if (rc) return rc;
    vecchia_graph* g = nullptr;
    try {
        g = begin_graph(x, n, d, k, n0, threads_of(n_threads));
        auto t0 = std::chrono::steady_clock::now();
        build_neighbours(*g, g->nthreads);
        g->times[1] = seconds_since(t0);
        finish_graph(*g);
    } catch (const std::bad_alloc&) {
        delete g;
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_build: host allocation failed (N=%lld, k=%d)", (long long)n, k);
    }
    *out = g;
    return VECCHIA_OK;
}

extern "C" int graph_build_begin(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0, int32_t n_threads,
                                 vecchia_graph** out) {
    vecchia_clear_error();
    int rc = check_build_args(x, n, d, k, n0, out, "graph_build_begin");
    if (rc) return rc;
    vecchia_graph* g = nullptr;
    try {
        g = begin_graph(x, n, d, k, n0, threads_of(n_threads));
        g->pending = true;
    } catch (const std::bad_alloc&) {
        delete g;
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_build_begin: host allocation failed (N=%lld)", (long long)n);
    }
    *out = g;
    return VECCHIA_OK;
}

extern "C" int graph_build_begin_tree(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0,
                                      int32_t n_threads, const int32_t* tree_perm, const int32_t* sdim,
                                      vecchia_graph** out) {
    vecchia_clear_error();
    int rc = check_build_args(x, n, d, k, n0, out, "graph_build_begin_tree");
    if (rc) return rc;
    if (!tree_perm || !sdim) return vecchia_set_error(VECCHIA_EINVAL, "graph_build_begin_tree: NULL tree");
    vecchia_graph* g = nullptr;
    try {
        const int nthreads = threads_of(n_threads);
        auto t0 = std::chrono::steady_clock::now();
        const int64_t bad = check_tree(x, n, d, tree_perm, sdim, nthreads);
        if (bad >= 0)
            return vecchia_set_error(VECCHIA_EINVAL, "graph_build_begin_tree: slot %lld breaks the tree of the points "
                                     "(permutation, split dimension or median order)", (long long)bad);
        g = new vecchia_graph();
        g->n = n;
        g->d = d;
        g->k = k;
        g->kp = vecchia_padded_k(k);
        g->n0 = n0;
        g->nthreads = nthreads;
        g->tree_perm.assign(tree_perm, tree_perm + n);
        g->sdim.resize(n);
        for (int64_t t = 0; t < n; ++t) g->sdim[t] = (int8_t)sdim[t];
        g->xs.resize((size_t)n * 3);
        parallel_for(n, 1 << 16, nthreads, [&](int64_t a, int64_t b) {
            for (int64_t t = a; t < b; ++t) {
                const int64_t i = g->tree_perm[t];
                for (int c = 0; c < 3; ++c) g->xs[t * 3 + c] = c < d ? x[i * d + c] : 0.0;
            }
        });
        inorder(*g);
        g->times[0] = seconds_since(t0);
        g->pending = true;
    } catch (const std::bad_alloc&) {
        delete g;
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_build_begin_tree: host allocation failed (N=%lld)", (long long)n);
    }
    *out = g;
    return VECCHIA_OK;
}

extern "C" int graph_knn_nodes(const vecchia_graph* g, void* nodes, int32_t* rank_of) {
    if (!g || !nodes || !rank_of) return vecchia_set_error(VECCHIA_EINVAL, "graph_knn_nodes: NULL argument");
    KnnNode* out = static_cast<KnnNode*>(nodes);
    const int64_t n = g->n;
    parallel_for(n, 1 << 16, g->nthreads, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int64_t t = g->seq[r];
            KnnNode& nd = out[r];
            for (int c = 0; c < 3; ++c) nd.c[c] = g->xs[t * 3 + c];
            nd.slot = (int32_t)t;
            const int64_t l = left_child(t), rr = right_child(t);
            nd.left = l < n ? g->rank_of[l] : -1;
            nd.right = rr < n ? g->rank_of[rr] : -1;
            nd.sdim = g->sdim[t];
        }
    });
    std::memcpy(rank_of, g->rank_of.data(), (size_t)n * sizeof(int32_t));
    return VECCHIA_OK;
}

namespace {

int finish_with(vecchia_graph* g, const int32_t* rows, const int32_t* depth) {
    vecchia_clear_error();
    if (!g || !rows) return vecchia_set_error(VECCHIA_EINVAL, "graph_build_finish: NULL argument");
    if (!g->pending) return vecchia_set_error(VECCHIA_EINVAL, "graph_build_finish: graph is not pending");
    const int64_t ns = g->n - g->n0;
    const int k = g->k;
    // rows come from outside the builder: every entry must name a preceding
    // slot, rows ascend by key, and padding (-1) only fills the tail of the
    // rows of slots with fewer than k predecessors
    std::atomic<int64_t> first_bad(ns);      // smallest failing row, ns if none
    parallel_for(ns, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int64_t i = g->n0 + r;
            const int64_t want = std::min<int64_t>(k, i);
            const double* q = &g->xs[i * 3];
            double prev_d = -1.0;
            int32_t prev_j = -1;
            bool ok = true;
            for (int m = 0; m < k && ok; ++m) {
                const int32_t j = rows[r * k + m];
                if (m < want ? (j < 0 || j >= i) : (j != -1)) ok = false;
                if (!ok || j < 0) continue;
                const double dd = sqdist(q, &g->xs[(int64_t)j * 3], g->d);
                if (m > 0 && !(dd > prev_d || (dd == prev_d && j > prev_j))) ok = false;
                prev_d = dd;
                prev_j = j;
            }
            if (!ok) {
                int64_t cur = first_bad.load();
                while (r < cur && !first_bad.compare_exchange_weak(cur, r)) {
                }
            }
        }
    });
    if (first_bad.load() < ns)
        return vecchia_set_error(VECCHIA_EINVAL,
                                 "graph_build_finish: the row of slot %lld names a slot that does not precede it, is "
                                 "padded before its end, or is not ascending by (distance, slot)",
                                 (long long)(g->n0 + first_bad.load()));
    try {
        g->nbr.resize((size_t)ns * k);
        parallel_for(ns, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
            for (int64_t q = a * k; q < b * k; ++q) g->nbr[q] = rows[q] >= 0 ? g->rank_of[rows[q]] : -1;
        });
        if (depth) {
            // depths from outside the builder: the dense block at 0 and every
            // sparse slot one above its deepest neighbour (Sec. 2.2)
            std::atomic<int64_t> bad(g->n);
            parallel_for(g->n, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
                for (int64_t i = a; i < b; ++i) {
                    int32_t want = 0;
                    if (i >= g->n0) {
                        const int32_t* row = &rows[(i - g->n0) * k];
                        int32_t m = 0;
                        for (int q = 0; q < k && row[q] >= 0; ++q) m = std::max(m, depth[row[q]]);
                        want = m + 1;
                    }
                    if (depth[i] != want) {
                        int64_t cur = bad.load();
                        while (i < cur && !bad.compare_exchange_weak(cur, i)) {
                        }
                    }
                }
            });
            if (bad.load() < g->n)
                return vecchia_set_error(VECCHIA_EINVAL, "graph_build_finish_depth: the depth of slot %lld does not "
                                         "follow the recurrence", (long long)bad.load());
        }
        finish_graph(*g, depth);
    } catch (const std::bad_alloc&) {
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_build_finish: host allocation failed");
    }
    return VECCHIA_OK;
}

}  // namespace

extern "C" int graph_build_finish(vecchia_graph* g, const int32_t* rows) { return finish_with(g, rows, nullptr); }

extern "C" int graph_build_finish_depth(vecchia_graph* g, const int32_t* rows, const int32_t* depth) {
    if (!depth) return vecchia_set_error(VECCHIA_EINVAL, "graph_build_finish_depth: depth is NULL");
    return finish_with(g, rows, depth);
}

extern "C" int graph_info(const vecchia_graph* g, int64_t* n, int32_t* d, int32_t* k, int32_t* kp, int32_t* n0,
                          int32_t* n_levels) {
    if (!g) return vecchia_set_error(VECCHIA_EINVAL, "graph_info: graph is NULL");
    if (n) *n = g->n;
    if (d) *d = g->d;
    if (k) *k = g->k;
    if (kp) *kp = g->kp;
    if (n0) *n0 = g->n0;
    if (n_levels) *n_levels = g->n_levels;
    return VECCHIA_OK;
}

extern "C" int graph_export(const vecchia_graph* g, int32_t* order, int32_t* slot, int32_t* level_ptr,
                            int32_t* depth) {
    if (g && g->pending) return vecchia_set_error(VECCHIA_EINVAL, "graph_export: the graph is pending (graph_build_finish)");
    if (!g) return vecchia_set_error(VECCHIA_EINVAL, "graph_export: graph is NULL");
    parallel_for(g->n, 1 << 16, g->nthreads, [&](int64_t a, int64_t b) {
        for (int64_t s = a; s < b; ++s) {
            const int32_t t = g->order[s];
            if (order) order[s] = g->tree_perm[t];
            if (slot) slot[s] = t;
            if (depth) depth[s] = g->depth[t];
        }
    });
    if (level_ptr) std::memcpy(level_ptr, g->level_ptr.data(), sizeof(int32_t) * g->level_ptr.size());
    return VECCHIA_OK;
}

extern "C" int graph_export_nbr(const vecchia_graph* g, int32_t layout, int32_t* nbr) {
    if (g && g->pending) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_nbr: the graph is pending (graph_build_finish)");
    if (!g || !nbr) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_nbr: NULL argument");
    if (layout != 0 && layout != 1) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_nbr: layout must be 0 or 1");
    const int64_t ns = g->n - g->n0;
    const int k = g->k, kp = g->kp;
    if (layout == 0) {
        parallel_for(ns, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
            for (int64_t sp = a; sp < b; ++sp) {
                const int32_t t = g->order[g->n0 + sp];
                const int32_t* row = &g->nbr[(size_t)(t - g->n0) * k];
                for (int m = 0; m < k; ++m) nbr[sp * k + m] = row[m] >= 0 ? g->pos_r[row[m]] : -1;
            }
        });
        return VECCHIA_OK;
    }
    const int64_t tiles = (ns + 63) / 64;
    parallel_for(tiles, 1024, g->nthreads, [&](int64_t a, int64_t b) {
        int32_t row[VECCHIA_KMAX];
        for (int64_t tile = a; tile < b; ++tile)
            for (int lane = 0; lane < 64; ++lane) {
                const int64_t sp = tile * 64 + lane;
                if (sp < ns) device_row(*g, sp, row);
                for (int m = 0; m < kp; ++m) nbr[(tile * kp + m) * 64 + lane] = (sp < ns && m < k) ? row[m] : -1;
            }
    });
    return VECCHIA_OK;
}

extern "C" int graph_export_points(const vecchia_graph* g, int32_t precision, void* xs) {
    if (g && g->pending) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_points: the graph is pending (graph_build_finish)");
    if (!g || !xs) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_points: NULL argument");
    if (precision != VECCHIA_FP64 && precision != VECCHIA_FP32)
        return vecchia_set_error(VECCHIA_EINVAL, "graph_export_points: bad precision %d", precision);
    parallel_for(g->n, 1 << 16, g->nthreads, [&](int64_t a, int64_t b) {
        for (int64_t s = a; s < b; ++s) {
            const double* p = &g->xs[(size_t)g->order[s] * 3];
            for (int c = 0; c < 3; ++c) {
                if (precision == VECCHIA_FP64)
                    static_cast<double*>(xs)[s * 3 + c] = p[c];
                else
                    static_cast<float*>(xs)[s * 3 + c] = (float)p[c];
            }
        }
    });
    return VECCHIA_OK;
}

extern "C" int graph_export_children(const vecchia_graph* g, int64_t* child_ptr, int32_t* child) {
    if (g && g->pending) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_children: the graph is pending (graph_build_finish)");
    if (!g || !child_ptr || !child) return vecchia_set_error(VECCHIA_EINVAL, "graph_export_children: NULL argument");
    const int64_t ns = g->n - g->n0;
    if (ns * g->kp >= (int64_t(1) << 31))
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "graph_export_children: Ns*kp = %lld does not fit int32", (long long)(ns * g->kp));
    // Counts and placement run in parallel with atomic per-list cursors, so
    // the order inside a list depends on the threads; each list is sorted
    // afterwards.  Its entries sp * kp + m are distinct and a row names a
    // point at most once, so the sorted list is the list in row order.
    std::vector<int64_t> cnt(g->n + 1, 0);
    int64_t* c = cnt.data();
    parallel_for(ns, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
        for (int64_t sp = a; sp < b; ++sp) {
            const int32_t t = g->order[g->n0 + sp];
            const int32_t* row = &g->nbr[(size_t)(t - g->n0) * g->k];
            for (int m = 0; m < g->k; ++m)
                if (row[m] >= 0) __atomic_fetch_add(&c[g->pos_r[row[m]] + 1], int64_t(1), __ATOMIC_RELAXED);
        }
    });
    for (int64_t j = 0; j < g->n; ++j) cnt[j + 1] += cnt[j];
    std::memcpy(child_ptr, cnt.data(), sizeof(int64_t) * (g->n + 1));
    parallel_for(ns, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
        int32_t row[VECCHIA_KMAX];
        for (int64_t sp = a; sp < b; ++sp) {
            device_row(*g, sp, row);                   // m: position in the device row
            for (int m = 0; m < g->k; ++m)
                if (row[m] >= 0) child[__atomic_fetch_add(&c[row[m]], int64_t(1), __ATOMIC_RELAXED)] = (int32_t)(sp * g->kp + m);
        }
    });
    parallel_for(g->n, 1 << 14, g->nthreads, [&](int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j) std::sort(child + child_ptr[j], child + child_ptr[j + 1]);
    });
    return VECCHIA_OK;
}

extern "C" int graph_build_times(const vecchia_graph* g, double* times) {
    if (!g || !times) return vecchia_set_error(VECCHIA_EINVAL, "graph_build_times: NULL argument");
    for (int i = 0; i < 4; ++i) times[i] = g->times[i];
    return VECCHIA_OK;
}

extern "C" void graph_free(vecchia_graph* g) { delete g; }
