// Serving engine: continuous batching of Vecchia requests on one GPU.
//
// A request carries its own point set, kernel parameters and one operation
// (forward, inverse or logdet).  Life cycle:
//   submit     -> copied to the host, queued for a graph worker
//   building   -> a worker thread runs graph_build and fills pinned staging
//                 buffers (coordinates, tiled neighbours, input in storage order)
//   queued     -> waits for admission: FIFO, admitted when its whole device
//                 footprint fits in the free part of the HBM arena
//   running    -> on one of the engine's streams: upload, vecchia_factor, the
//                 operation, download, completion event
//   done       -> the arena range is freed at completion; the result stays on
//                 the host until serve_release
// Requests of different size and k run concurrently on different streams, so
// work that arrives while others are on the GPU overlaps with them.  The
// device memory is one buffer owned by the caller (the budget); this file only
// carves it (first-fit free list, 256-byte aligned, coalescing frees).
//
// Mock mode runs the same scheduler with no device calls (the operation
// "finishes" after a fixed number of serve_progress calls), for host tests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "status.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, cap) with coalescing.
class Arena {
public:
    explicit Arena(size_t cap) : cap_(cap) { free_[0] = cap; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = vk::align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = vk::align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t cap() const { return cap_; }
    size_t largest_free() const {
        size_t m = 0;
        for (auto& f : free_) m = std::max(m, f.second);
        return m;
    }

private:
    size_t cap_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum State { BUILDING = 0, QUEUED = 1, RUNNING = 2, DONE = 3, FAILED = 4, CANCELLED = 5 };

struct Footprint {
    size_t x = 0, nbr = 0, ws = 0, in = 0, out = 0, ld = 0, lp = 0, total = 0;
};

// Device bytes of one request with n_levels batches (n - n0 is an upper bound
// before the graph is built).
Footprint footprint(int64_t n, int kp, int n0, int64_t n_levels) {
    Footprint f;
    const int64_t ns = n - n0;
    const int64_t tiles = (ns + 63) / 64;
    size_t off = 0;
    f.x = off;
    off = vk::align256(off + (size_t)n * 3 * sizeof(float));
    f.nbr = off;
    off = vk::align256(off + (size_t)std::max<int64_t>(tiles, 1) * kp * 64 * sizeof(int32_t));
    f.ws = off;
    off = vk::align256(off + vk::workspace_layout(n, kp, n0, VECCHIA_FP32).total);
    f.in = off;
    off = vk::align256(off + (size_t)n * sizeof(float));
    f.out = off;
    off = vk::align256(off + (size_t)n * sizeof(float));
    f.ld = off;
    off = vk::align256(off + sizeof(double));
    f.lp = off;
    off = vk::align256(off + (size_t)(n_levels + 2) * sizeof(int32_t));
    f.total = off;
    return f;
}

struct Request {
    int64_t id = 0;
    int op = 0, k = 0, kp = 0, n0 = 0;
    int64_t n = 0;
    vecchia_kernel kern{};
    std::vector<double> x;        // input order, n x 3
    std::vector<float> input;     // input order, n (forward/inverse)
    std::atomic<int> state{BUILDING};
    bool in_build = false;        // a worker holds this request (guarded by the server mutex)
    int status = VECCHIA_OK;
    std::string error;
    // graph products
    int n_levels = 0;
    std::vector<int32_t> order, level_ptr;
    void* h_block = nullptr;       // one page-locked allocation holding the six staging arrays (GPU mode)
    float* h_x = nullptr;          // pinned staging, carved from h_block
    int32_t* h_nbr = nullptr;
    float* h_in = nullptr;
    float* h_out = nullptr;
    double* h_ld = nullptr;
    int32_t* h_lp = nullptr;
    std::vector<float> mock_out;
    // device
    Footprint fp;
    size_t arena_off = 0;
    int stream = -1;
    hipEvent_t done_ev = nullptr;
    vecchia_view view{};
    int mock_ticks = 0;
    // timestamps
    double t_submit = 0, t_graph = 0, t_admit = 0, t_done = 0;
};

void free_pinned(Request& r) {
    if (r.h_block) (void)hipHostFree(r.h_block);
    r.h_block = nullptr;
    r.h_lp = nullptr;
    r.h_x = nullptr;
    r.h_nbr = nullptr;
    r.h_in = r.h_out = nullptr;
    r.h_ld = nullptr;
}

}  // namespace

struct vecchia_server {
    char* base = nullptr;
    std::unique_ptr<Arena> arena;
    bool mock = false;
    int mock_latency = 3;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    int graph_threads = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request*> build_q;
    std::deque<Request*> ready_q;      // graph done, waiting for admission (FIFO)
    std::vector<Request*> running;
    std::deque<int64_t> completed;     // ids not yet taken
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::vector<std::thread> workers;
    bool stop = false;
    int64_t next_id = 1;
    int64_t n_admitted = 0, n_done = 0, n_failed = 0, n_rejected = 0, n_cancelled = 0;
    int64_t peak_running = 0;   // most requests on the device at once
    // device graph builds (serve_set_graph_device): one slice and one stream per worker
    char* gdev = nullptr;
    size_t gslice = 0;
    std::vector<hipStream_t> wstreams;
    int64_t n_graph_device = 0;  // graphs built through the device path
};

namespace {

// Graphs below this size are built on the host: the device path's fixed
// costs (transfers, a synchronisation per step) exceed their build time.
constexpr int64_t kDeviceGraphMin = int64_t(1) << 15;

// Bytes of a worker's slice that the device build of n points needs: the
// tree phase (coordinates, sort scratch, tree) and, reusing the same bytes,
// the neighbour phase (nodes, ranks, rows, depths, a flag).
size_t device_graph_bytes(int64_t n, int k, int n0) {
    size_t tree = 0;
    if (graph_tree_scratch_bytes(n, &tree) != VECCHIA_OK) return ~size_t(0);
    const size_t a = vk::align256((size_t)n * 24) + vk::align256(tree) + 2 * vk::align256((size_t)n * 4);
    const size_t b = vk::align256((size_t)n * VECCHIA_KNN_NODE_BYTES) + vk::align256((size_t)n * 4) +
                     vk::align256((size_t)std::max<int64_t>(n - n0, 1) * k * 4) + vk::align256((size_t)n * 4) + 256;
    return std::max(a, b);
}

// The graph through the device steps (tree, neighbour search, depths) in the
// worker's slice, on its stream; the host checks each step's result as in
// the split build.  Same graph as graph_build, bit for bit.
int build_graph_device(vecchia_server* s, int wid, Request* r, int threads, vecchia_graph** out) {
    char* d = s->gdev + (size_t)wid * s->gslice;
    hipStream_t st = s->wstreams[wid];
    const int64_t n = r->n;
    const int k = r->k, n0 = r->n0;
    size_t tb = 0;
    int rc = graph_tree_scratch_bytes(n, &tb);
    if (rc) return rc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = d + off;
        off += vk::align256(bytes);
        return p;
    };
    double* dx = reinterpret_cast<double*>(take((size_t)n * 24));
    void* scr = take(tb);
    int32_t* dperm = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    int32_t* dsdim = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    std::vector<int32_t> perm(n), sdim(n);
    // an error return drains the worker's stream first: copies into this
    // function's host vectors may still be queued on it
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(st);
        return code;
    };
    hipError_t e = hipMemcpyAsync(dx, r->x.data(), (size_t)n * 24, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(vecchia_set_error(VECCHIA_EHIP, "serve graph upload: %s", hipGetErrorString(e)));
    if ((rc = graph_tree_device(dx, n, 3, dperm, dsdim, scr, tb, st))) return fail(rc);
    e = hipMemcpyAsync(perm.data(), dperm, (size_t)n * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sdim.data(), dsdim, (size_t)n * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(vecchia_set_error(VECCHIA_EHIP, "serve graph tree: %s", hipGetErrorString(e)));
    vecchia_graph* g = nullptr;
    if ((rc = graph_build_begin_tree(r->x.data(), n, 3, k, n0, threads, perm.data(), sdim.data(), &g))) return rc;
    std::vector<uint8_t> nodes((size_t)n * VECCHIA_KNN_NODE_BYTES);
    std::vector<int32_t> rank(n), depth(n), rows((size_t)std::max<int64_t>(n - n0, 1) * k);
    if ((rc = graph_knn_nodes(g, nodes.data(), rank.data()))) {
        graph_free(g);
        return rc;
    }
    off = 0;                                            // the tree phase's bytes are free again
    void* dnodes = take(nodes.size());
    int32_t* drank = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    int32_t* drows = reinterpret_cast<int32_t*>(take(rows.size() * 4));
    int32_t* ddepth = reinterpret_cast<int32_t*>(take((size_t)n * 4));
    int32_t* dflag = reinterpret_cast<int32_t*>(take(4));
    e = hipMemcpyAsync(dnodes, nodes.data(), nodes.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(drank, rank.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) rc = vecchia_set_error(VECCHIA_EHIP, "serve graph nodes: %s", hipGetErrorString(e));
    if (!rc) rc = graph_knn_device(dnodes, drank, n, 3, k, n0, drows, st);
    int32_t sweeps = 0;
    if (!rc) rc = graph_depth_device(drows, n, k, n0, ddepth, dflag, st, &sweeps);
    if (!rc) {
        e = hipMemcpyAsync(rows.data(), drows, rows.size() * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(depth.data(), ddepth, (size_t)n * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = vecchia_set_error(VECCHIA_EHIP, "serve graph rows: %s", hipGetErrorString(e));
    }
    if (!rc) rc = graph_build_finish_depth(g, rows.data(), depth.data());
    if (rc) {
        graph_free(g);
        return fail(rc);
    }
    *out = g;
    return VECCHIA_OK;
}

void build_request(vecchia_server* s, Request* r, int wid) {
    vecchia_graph* g = nullptr;
    const int threads = (int)std::max<int64_t>(1, std::min<int64_t>(s->graph_threads, r->n >> 16));
    char* gdev;
    size_t gslice;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        gdev = s->gdev;
        gslice = s->gslice;
    }
    int rc;
    if (gdev && r->n >= kDeviceGraphMin && device_graph_bytes(r->n, r->k, r->n0) <= gslice) {
        rc = build_graph_device(s, wid, r, threads, &g);
        std::lock_guard<std::mutex> lk(s->mu);
        if (rc == VECCHIA_OK) s->n_graph_device++;
    } else {
        rc = graph_build(r->x.data(), r->n, 3, r->k, r->n0, threads, &g);
    }
    if (rc == VECCHIA_OK) {
        graph_info(g, nullptr, nullptr, nullptr, nullptr, nullptr, &r->n_levels);
        r->order.resize(r->n);
        r->level_ptr.resize(r->n_levels + 2);
        graph_export(g, r->order.data(), nullptr, r->level_ptr.data(), nullptr);
        r->fp = footprint(r->n, r->kp, r->n0, r->n_levels);
        const int64_t tiles = std::max<int64_t>((r->n - r->n0 + 63) / 64, 1);
        if (!s->mock) {
            // one page-locked block per request (a page-locking call costs far
            // more than carving), each array at a 256-byte boundary
            auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
            const size_t bx = up((size_t)r->n * 3 * sizeof(float)), bn = up((size_t)tiles * r->kp * 64 * sizeof(int32_t));
            const size_t bv = up((size_t)r->n * sizeof(float)), bd = up(sizeof(double));
            const size_t bl = up((size_t)(r->n_levels + 2) * sizeof(int32_t));
            hipError_t e = hipHostMalloc(&r->h_block, bx + bn + 2 * bv + bd + bl, hipHostMallocDefault);
            if (e == hipSuccess) {
                char* base = static_cast<char*>(r->h_block);
                r->h_x = reinterpret_cast<float*>(base);
                r->h_nbr = reinterpret_cast<int32_t*>(base + bx);
                r->h_in = reinterpret_cast<float*>(base + bx + bn);
                r->h_out = reinterpret_cast<float*>(base + bx + bn + bv);
                r->h_ld = reinterpret_cast<double*>(base + bx + bn + 2 * bv);
                r->h_lp = reinterpret_cast<int32_t*>(base + bx + bn + 2 * bv + bd);
            } else {
                r->h_block = nullptr;
            }
            if (e != hipSuccess) {
                rc = VECCHIA_ENOMEM;
                r->error = std::string("pinned staging: ") + hipGetErrorString(e);
            } else {
                std::fill(r->h_nbr, r->h_nbr + (size_t)tiles * r->kp * 64, -1);
                std::memcpy(r->h_lp, r->level_ptr.data(), (size_t)(r->n_levels + 2) * sizeof(int32_t));
                graph_export_points(g, VECCHIA_FP32, r->h_x);
                if (r->n > r->n0) graph_export_nbr(g, 1, r->h_nbr);
                if (!r->input.empty())
                    for (int64_t s2 = 0; s2 < r->n; ++s2) r->h_in[s2] = r->input[r->order[s2]];
            }
        }
        graph_free(g);
    } else {
        r->error = vecchia_last_error();
    }
    r->x.clear();
    r->x.shrink_to_fit();
    r->t_graph = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    r->in_build = false;
    if (r->state.load() == CANCELLED) return;
    if (rc != VECCHIA_OK) {
        r->status = rc;
        r->state = FAILED;
        s->completed.push_back(r->id);
        s->n_failed++;
        return;
    }
    r->state = QUEUED;
    s->ready_q.push_back(r);
}

void worker_main(vecchia_server* s, int wid) {
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->build_q.empty(); });
            if (s->stop) return;
            r = s->build_q.front();
            s->build_q.pop_front();
            if (r->state.load() == CANCELLED) continue;
            r->in_build = true;
        }
        build_request(s, r, wid);
    }
}

// Enqueue upload + factor + operation + download on the request's stream.
int launch_request(vecchia_server* s, Request* r) {
    hipStream_t st = s->streams[r->stream];
    char* d = s->base + r->arena_off;
    const Footprint& f = r->fp;
    const int64_t tiles = std::max<int64_t>((r->n - r->n0 + 63) / 64, 1);
    hipError_t e = hipMemcpyAsync(d + f.x, r->h_x, (size_t)r->n * 3 * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d + f.nbr, r->h_nbr, (size_t)tiles * r->kp * 64 * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && r->op != VECCHIA_OP_LOGDET)
        e = hipMemcpyAsync(d + f.in, r->h_in, (size_t)r->n * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d + f.lp, r->h_lp, (size_t)(r->n_levels + 2) * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return vecchia_set_error(VECCHIA_EHIP, "serve upload: %s", hipGetErrorString(e));
    vecchia_view& v = r->view;
    v.n = r->n;
    v.k = r->k;
    v.kp = r->kp;
    v.n0 = r->n0;
    v.n_levels = r->n_levels;
    v.precision = VECCHIA_FP32;
    v.redo_log2 = 0;
    v.x = d + f.x;
    v.nbr = reinterpret_cast<const int32_t*>(d + f.nbr);
    v.level_ptr = r->level_ptr.data();
    v.level_ptr_dev = reinterpret_cast<const int32_t*>(d + f.lp);
    v.child_ptr = nullptr;
    v.child = nullptr;
    v.workspace = d + f.ws;
    v.workspace_bytes = vk::workspace_layout(r->n, r->kp, r->n0, VECCHIA_FP32).total;
    int rc = vecchia_factor(&v, &r->kern, st);
    if (rc) return rc;
    if (r->op == VECCHIA_OP_FORWARD) rc = vecchia_forward(&v, d + f.in, d + f.out, st);
    else if (r->op == VECCHIA_OP_INVERSE) rc = vecchia_inverse(&v, d + f.in, d + f.out, st);
    else rc = vecchia_logdet(&v, reinterpret_cast<double*>(d + f.ld), st);
    if (rc) return rc;
    if (r->op == VECCHIA_OP_LOGDET)
        e = hipMemcpyAsync(r->h_ld, d + f.ld, sizeof(double), hipMemcpyDeviceToHost, st);
    else
        e = hipMemcpyAsync(r->h_out, d + f.out, (size_t)r->n * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && !r->done_ev) e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->done_ev, st);
    if (e != hipSuccess) return vecchia_set_error(VECCHIA_EHIP, "serve launch: %s", hipGetErrorString(e));
    return VECCHIA_OK;
}

void finish(vecchia_server* s, Request* r, int status) {
    r->t_done = now_s();
    r->status = status;
    r->state = status == VECCHIA_OK ? DONE : FAILED;
    s->arena->release(r->arena_off, r->fp.total);
    s->stream_load[r->stream]--;
    s->completed.push_back(r->id);
    if (status == VECCHIA_OK)
        s->n_done++;
    else
        s->n_failed++;
}

}  // namespace

extern "C" int serve_create(void* arena, size_t arena_bytes, int32_t n_streams, int32_t graph_workers,
                            int32_t graph_threads, int32_t mock, vecchia_server** out) {
    vecchia_clear_error();
    if (!out) return vecchia_set_error(VECCHIA_EINVAL, "serve_create: out is NULL");
    *out = nullptr;
    if ((!arena && !mock) || arena_bytes < 256 || (reinterpret_cast<uintptr_t>(arena) & 255))
        return vecchia_set_error(VECCHIA_EINVAL, "serve_create: arena must be a 256-byte aligned buffer");
    if (n_streams < 1 || n_streams > 64 || graph_workers < 1 || graph_workers > 256)
        return vecchia_set_error(VECCHIA_EINVAL, "serve_create: need 1..64 streams and 1..256 graph workers");
    auto* s = new vecchia_server();
    s->base = static_cast<char*>(arena);
    s->arena.reset(new Arena(arena_bytes & ~size_t(255)));
    s->mock = mock != 0;
    s->graph_threads = std::max(1, (int)graph_threads);
    s->stream_load.assign(n_streams, 0);
    if (!s->mock) {
        s->streams.resize(n_streams);
        for (auto& st : s->streams) {
            hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                delete s;
                return vecchia_set_error(VECCHIA_EHIP, "serve_create: %s", hipGetErrorString(e));
            }
        }
    }
    if (!s->mock) {
        s->wstreams.resize(graph_workers);
        for (auto& st : s->wstreams) {
            hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (auto& q : s->streams) (void)hipStreamDestroy(q);
                delete s;
                return vecchia_set_error(VECCHIA_EHIP, "serve_create: %s", hipGetErrorString(e));
            }
        }
    }
    for (int w = 0; w < graph_workers; ++w) s->workers.emplace_back(worker_main, s, w);
    *out = s;
    return VECCHIA_OK;
}

extern "C" int serve_set_graph_device(vecchia_server* s, void* buffer, size_t bytes) {
    vecchia_clear_error();
    if (!s) return vecchia_set_error(VECCHIA_EINVAL, "serve_set_graph_device: server is NULL");
    if (s->mock) return vecchia_set_error(VECCHIA_EINVAL, "serve_set_graph_device: a mock server has no device");
    if (buffer && (reinterpret_cast<uintptr_t>(buffer) & 255))
        return vecchia_set_error(VECCHIA_EINVAL, "serve_set_graph_device: buffer must be 256-byte aligned");
    std::lock_guard<std::mutex> lk(s->mu);
    s->gdev = static_cast<char*>(buffer);
    s->gslice = buffer ? (bytes / s->workers.size()) & ~size_t(255) : 0;
    return VECCHIA_OK;
}

extern "C" int serve_request_bytes(int64_t n, int32_t k, int32_t n0, size_t* bytes) {
    if (k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "serve_request_bytes: k=%d exceeds the compiled maximum %d", k,
                                 VECCHIA_KMAX);
    const int kp = vecchia_padded_k(k);
    if (!bytes || kp < 0 || n < 1 || n0 < 1 || n0 > n)
        return vecchia_set_error(VECCHIA_EINVAL, "serve_request_bytes: bad arguments");
    *bytes = footprint(n, kp, n0, n - n0).total;
    return VECCHIA_OK;
}

extern "C" int serve_submit(vecchia_server* s, const double* x, int64_t n, int32_t k, int32_t n0,
                            const vecchia_kernel* kern, int32_t op, const float* input, int64_t* id) {
    vecchia_clear_error();
    if (!s || !x || !kern || !id) return vecchia_set_error(VECCHIA_EINVAL, "serve_submit: NULL argument");
    if (op < VECCHIA_OP_FORWARD || op > VECCHIA_OP_LOGDET)
        return vecchia_set_error(VECCHIA_EINVAL, "serve_submit: op must be forward, inverse or logdet");
    if (op != VECCHIA_OP_LOGDET && !input) return vecchia_set_error(VECCHIA_EINVAL, "serve_submit: input is NULL");
    if (k > VECCHIA_KMAX || n0 > VECCHIA_N0MAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "serve_submit: k=%d or n0=%d exceeds the compiled maximum (%d, %d)",
                                 k, n0, VECCHIA_KMAX, VECCHIA_N0MAX);
    const int kp = vecchia_padded_k(k);
    if (kp < 0 || n < 1 || n >= (int64_t(1) << 31) || n0 < 1 || n0 > n)
        return vecchia_set_error(VECCHIA_EINVAL, "serve_submit: need 1 <= k <= %d and 1 <= n0 <= min(N, %d)",
                                 VECCHIA_KMAX, VECCHIA_N0MAX);
    if (kern->kind < 0 || kern->kind > 3 || !(kern->sigma > 0) || !(kern->ell > 0) || !(kern->nugget >= 0))
        return vecchia_set_error(VECCHIA_EINVAL, "serve_submit: bad kernel parameters");
    const Footprint fp = footprint(n, kp, n0, n - n0);   // exact size once the graph is built
    std::unique_ptr<Request> r(new Request());
    r->fp = fp;
    std::lock_guard<std::mutex> lk(s->mu);
    if (fp.total > s->arena->cap()) {
        s->n_rejected++;
        return vecchia_set_error(VECCHIA_EBUDGET, "serve_submit: request needs %zu bytes, the arena holds %zu",
                                 fp.total, s->arena->cap());
    }
    r->id = s->next_id++;
    r->op = op;
    r->k = k;
    r->kp = kp;
    r->n = n;
    r->n0 = n0;
    r->kern = *kern;
    r->x.assign(x, x + n * 3);
    if (op != VECCHIA_OP_LOGDET) r->input.assign(input, input + n);
    r->t_submit = now_s();
    *id = r->id;
    s->build_q.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    s->cv.notify_one();
    return VECCHIA_OK;
}

extern "C" int serve_progress(vecchia_server* s, int32_t* n_completed) {
    vecchia_clear_error();
    if (!s) return vecchia_set_error(VECCHIA_EINVAL, "serve_progress: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    int first_error = VECCHIA_OK;
    // completions
    for (size_t i = 0; i < s->running.size();) {
        Request* r = s->running[i];
        bool done = false;
        if (s->mock) {
            done = ++r->mock_ticks >= s->mock_latency;
        } else {
            hipError_t e = hipEventQuery(r->done_ev);
            if (e == hipSuccess) done = true;
            else if (e != hipErrorNotReady) {
                finish(s, r, vecchia_set_error(VECCHIA_EHIP, "serve request %lld: %s", (long long)r->id,
                                               hipGetErrorString(e)));
                first_error = first_error ? first_error : VECCHIA_EHIP;
                s->running.erase(s->running.begin() + i);
                continue;
            }
        }
        if (done) {
            if (s->mock && r->op != VECCHIA_OP_LOGDET) r->mock_out.assign(r->input.begin(), r->input.end());
            finish(s, r, VECCHIA_OK);
            s->running.erase(s->running.begin() + i);
        } else {
            ++i;
        }
    }
    // admissions: FIFO while the head fits
    while (!s->ready_q.empty()) {
        Request* r = s->ready_q.front();
        if (r->state.load() == CANCELLED) {
            s->ready_q.pop_front();
            continue;
        }
        size_t off = 0;
        if (!s->arena->alloc(r->fp.total, &off)) break;
        s->ready_q.pop_front();
        r->arena_off = off;
        r->t_admit = now_s();
        int best = 0;
        for (int i = 1; i < (int)s->stream_load.size(); ++i)
            if (s->stream_load[i] < s->stream_load[best]) best = i;
        r->stream = best;
        s->stream_load[best]++;
        r->state = RUNNING;
        s->n_admitted++;
        if (!s->mock) {
            const int rc = launch_request(s, r);
            if (rc) {
                r->error = vecchia_last_error();
                // part of the request's work may already be queued on its
                // stream and still use its arena range: let it drain before
                // finish() hands the range to the next request
                (void)hipStreamSynchronize(s->streams[r->stream]);
                finish(s, r, rc);
                first_error = first_error ? first_error : rc;
                continue;
            }
        }
        s->running.push_back(r);
        s->peak_running = std::max<int64_t>(s->peak_running, (int64_t)s->running.size());
    }
    if (n_completed) *n_completed = (int32_t)s->completed.size();
    return first_error;
}

extern "C" int serve_take(vecchia_server* s, int64_t* id) {
    if (!s || !id) return vecchia_set_error(VECCHIA_EINVAL, "serve_take: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->completed.empty()) {
        *id = 0;
        return VECCHIA_OK;
    }
    *id = s->completed.front();
    s->completed.pop_front();
    return VECCHIA_OK;
}

extern "C" int serve_result(vecchia_server* s, int64_t id, float* out, double* logdet, double* times) {
    vecchia_clear_error();
    if (!s) return vecchia_set_error(VECCHIA_EINVAL, "serve_result: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return vecchia_set_error(VECCHIA_EINVAL, "serve_result: unknown request %lld", (long long)id);
    Request* r = it->second.get();
    const int st = r->state.load();
    if (st != DONE && st != FAILED)
        return vecchia_set_error(VECCHIA_EINVAL, "serve_result: request %lld not finished", (long long)id);
    if (times) {
        times[0] = r->t_graph - r->t_submit;
        times[1] = st == DONE || r->t_admit > 0 ? r->t_admit - r->t_graph : 0.0;
        times[2] = r->t_admit > 0 ? r->t_done - r->t_admit : 0.0;
        times[3] = (r->t_done > 0 ? r->t_done : r->t_graph) - r->t_submit;
    }
    if (st == FAILED) return vecchia_set_error(r->status ? r->status : VECCHIA_EINVAL, "request %lld failed: %s",
                                               (long long)id, r->error.c_str());
    if (r->op == VECCHIA_OP_LOGDET) {
        if (logdet) *logdet = s->mock ? 0.0 : *r->h_ld;
    } else if (out) {
        if (s->mock) {
            std::memcpy(out, r->mock_out.data(), sizeof(float) * r->n);
        } else {
            for (int64_t p = 0; p < r->n; ++p) out[r->order[p]] = r->h_out[p];   // back to input order
        }
    }
    return VECCHIA_OK;
}

extern "C" int serve_release(vecchia_server* s, int64_t id) {
    if (!s) return vecchia_set_error(VECCHIA_EINVAL, "serve_release: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return vecchia_set_error(VECCHIA_EINVAL, "serve_release: unknown request");
    Request* r = it->second.get();
    const int st = r->state.load();
    if ((st != DONE && st != FAILED && st != CANCELLED) || r->in_build)
        return vecchia_set_error(VECCHIA_EINVAL, "serve_release: request %lld still in flight", (long long)id);
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);
    free_pinned(*r);
    s->reqs.erase(it);
    return VECCHIA_OK;
}

extern "C" int serve_cancel(vecchia_server* s, int64_t id) {
    if (!s) return vecchia_set_error(VECCHIA_EINVAL, "serve_cancel: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return vecchia_set_error(VECCHIA_EINVAL, "serve_cancel: unknown request");
    Request* r = it->second.get();
    int expected = QUEUED;
    if (r->state.compare_exchange_strong(expected, CANCELLED) ||
        (expected = BUILDING, r->state.compare_exchange_strong(expected, CANCELLED))) {
        // Drop every queue's pointer to it now, under the mutex, so that
        // serve_release may free it at once: a worker that already holds it
        // (in_build) sees CANCELLED when it finishes and queues nothing.
        s->build_q.erase(std::remove(s->build_q.begin(), s->build_q.end(), r), s->build_q.end());
        s->ready_q.erase(std::remove(s->ready_q.begin(), s->ready_q.end(), r), s->ready_q.end());
        s->n_cancelled++;
        return VECCHIA_OK;
    }
    return vecchia_set_error(VECCHIA_EINVAL, "serve_cancel: request %lld is already running or finished", (long long)id);
}

extern "C" int serve_stats(vecchia_server* s, vecchia_serve_stats* out) {
    if (!s || !out) return vecchia_set_error(VECCHIA_EINVAL, "serve_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t building = 0, queued = 0;
    for (auto& kv : s->reqs) {
        const int st = kv.second->state.load();
        building += st == BUILDING;
        queued += st == QUEUED;
    }
    out->arena_bytes = s->arena->cap();
    out->bytes_in_use = s->arena->used();
    out->peak_bytes = s->arena->peak();
    out->largest_free = s->arena->largest_free();
    out->building = building;
    out->queued = queued;
    out->running = (int64_t)s->running.size();
    out->admitted = s->n_admitted;
    out->completed = s->n_done;
    out->failed = s->n_failed;
    out->rejected = s->n_rejected;
    out->cancelled = s->n_cancelled;
    out->peak_running = s->peak_running;
    out->graphs_on_device = s->n_graph_device;
    return VECCHIA_OK;
}

extern "C" void serve_destroy(vecchia_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (auto& t : s->workers) t.join();
    if (!s->mock) {
        for (auto& st : s->streams) (void)hipStreamSynchronize(st);
    }
    for (auto& kv : s->reqs) {
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
        free_pinned(*kv.second);
    }
    for (auto& st : s->wstreams) (void)hipStreamSynchronize(st);
    for (auto& st : s->streams) (void)hipStreamDestroy(st);
    for (auto& st : s->wstreams) (void)hipStreamDestroy(st);
    delete s;
}
