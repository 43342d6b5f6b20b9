// Host-only driver for the sanitizer builds of the graph builder and of the
// serving scheduler in mock mode (no device calls).  Built by
// tests/test_sanitizers.py with AddressSanitizer + UndefinedBehaviorSanitizer
// and, separately, with ThreadSanitizer; any report fails the run.
//
// Scenarios: graph builds with every dimension and several widths and thread
// counts, including a padded dense-check row set, each saved to a graph file,
// loaded back and compared, and loaded again cut short; the scheduler with requests
// that complete, a request cancelled while it waits for memory, one cancelled
// while its graph is still being built, and both released at once after the
// cancel (the path that must not leave a queue pointing at freed memory).
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include <unistd.h>

#include "vecchia.h"

#define CHECK(cond)                                                                              \
    do {                                                                                         \
        if (!(cond)) {                                                                           \
            std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond,          \
                         vecchia_last_error());                                                  \
            std::exit(1);                                                                        \
        }                                                                                        \
    } while (0)

// The scheduler's device calls, never reached in mock mode: the sanitizer
// build links these instead of the HIP kernels.
extern "C" int vecchia_factor(vecchia_view*, const vecchia_kernel*, void*) { std::abort(); }
extern "C" int vecchia_forward(const vecchia_view*, const void*, void*, void*) { std::abort(); }
extern "C" int vecchia_inverse(const vecchia_view*, const void*, void*, void*) { std::abort(); }
extern "C" int vecchia_logdet(const vecchia_view*, double*, void*) { std::abort(); }
extern "C" int graph_tree_scratch_bytes(int64_t, size_t*) { std::abort(); }
extern "C" int graph_tree_device(const double*, int64_t, int32_t, int32_t*, int32_t*, void*, size_t, void*) {
    std::abort();
}
extern "C" int graph_knn_device(const void*, const int32_t*, int64_t, int32_t, int32_t, int32_t, int32_t*, void*) {
    std::abort();
}
extern "C" int graph_depth_device(const int32_t*, int64_t, int32_t, int32_t, int32_t*, int32_t*, void*, int32_t*) {
    std::abort();
}

static std::vector<double> points(int64_t n, int d, unsigned seed) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<double> x((size_t)n * d);
    for (auto& v : x) v = u(rng);
    return x;
}

static void graphs() {
    struct Case { int64_t n; int d, k, n0, threads; };
    const Case cases[] = {{3000, 3, 8, 128, 1}, {5000, 3, 32, 64, 4}, {2000, 2, 16, 32, 2},
                          {1500, 1, 5, 16, 3},  {65, 3, 32, 1, 2},   {300, 3, 8, 300, 1},
                          {40000, 3, 8, 64, 4}};   // last: several chunks per threaded pass
    for (const Case& c : cases) {
        std::vector<double> x = points(c.n, c.d, (unsigned)(c.n + c.k));
        vecchia_graph* g = nullptr;
        CHECK(graph_build(x.data(), c.n, c.d, c.k, c.n0, c.threads, &g) == VECCHIA_OK);
        int64_t n = 0;
        int32_t d = 0, k = 0, kp = 0, n0 = 0, levels = 0;
        CHECK(graph_info(g, &n, &d, &k, &kp, &n0, &levels) == VECCHIA_OK);
        std::vector<int32_t> order(n), slot(n), lp(levels + 2), depth(n);
        CHECK(graph_export(g, order.data(), slot.data(), lp.data(), depth.data()) == VECCHIA_OK);
        const int64_t ns = n - n0, tiles = (ns + 63) / 64;
        std::vector<int32_t> rows((size_t)std::max<int64_t>(ns * k, 1)), tiled((size_t)std::max<int64_t>(tiles * kp * 64, 1));
        CHECK(graph_export_nbr(g, 0, rows.data()) == VECCHIA_OK);
        CHECK(graph_export_nbr(g, 1, tiled.data()) == VECCHIA_OK);
        std::vector<float> xf((size_t)n * 3);
        CHECK(graph_export_points(g, VECCHIA_FP32, xf.data()) == VECCHIA_OK);
        std::vector<int64_t> cptr(n + 1);
        std::vector<int32_t> child((size_t)std::max<int64_t>(ns * k, 1));
        CHECK(graph_export_children(g, cptr.data(), child.data()) == VECCHIA_OK);
        CHECK(cptr[n] <= ns * k);
        for (int64_t s = 0; s < ns * k; ++s) CHECK(rows[s] < n0 + s / k);   // neighbours precede
        // graph file round trip, then the same file cut short
        char path[] = "/tmp/vecchia_graph_XXXXXX";
        const int fd = mkstemp(path);
        CHECK(fd >= 0);
        close(fd);
        CHECK(graph_save(g, path) == VECCHIA_OK);
        vecchia_graph* h = nullptr;
        CHECK(graph_load(path, c.threads, &h) == VECCHIA_OK);
        std::vector<int32_t> order2(n), rows2(rows.size());
        CHECK(graph_export(h, order2.data(), nullptr, nullptr, nullptr) == VECCHIA_OK);
        CHECK(graph_export_nbr(h, 0, rows2.data()) == VECCHIA_OK);
        CHECK(order2 == order && std::equal(rows2.begin(), rows2.begin() + ns * k, rows.begin()));
        graph_free(h);
        FILE* f = std::fopen(path, "r+b");
        CHECK(f && std::fseek(f, 0, SEEK_END) == 0);
        const long len = std::ftell(f);
        std::fclose(f);
        CHECK(truncate(path, len / 2) == 0);
        h = nullptr;
        CHECK(graph_load(path, c.threads, &h) == VECCHIA_EIO && h == nullptr);
        std::remove(path);
        graph_free(g);
    }
}

static void wait_built(vecchia_server* s) {
    for (int i = 0; i < 20000; ++i) {
        vecchia_serve_stats st;
        CHECK(serve_stats(s, &st) == VECCHIA_OK);
        if (st.building == 0) return;
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    CHECK(!"graph workers did not finish");
}

static void scheduler() {
    vecchia_kernel kern{1, 1.0, 0.1, 0.0};
    size_t one = 0;
    CHECK(serve_request_bytes(60000, 16, 128, &one) == VECCHIA_OK);
    vecchia_server* s = nullptr;
    CHECK(serve_create(nullptr, one + 1024, 2, 2, 2, 1, &s) == VECCHIA_OK);   // room for one request
    std::vector<double> x = points(60000, 3, 7);
    std::vector<float> in(60000, 1.0f);
    int64_t a = 0, b = 0, c = 0;
    CHECK(serve_submit(s, x.data(), 60000, 16, 128, &kern, VECCHIA_OP_FORWARD, in.data(), &a) == VECCHIA_OK);
    CHECK(serve_submit(s, x.data(), 60000, 16, 128, &kern, VECCHIA_OP_INVERSE, in.data(), &b) == VECCHIA_OK);
    wait_built(s);
    int32_t done = 0;
    CHECK(serve_progress(s, &done) == VECCHIA_OK);   // one of a, b admitted, the other waits for memory
    int64_t waiting = b;                              // (two workers: either graph may be ready first)
    if (serve_cancel(s, b) != VECCHIA_OK) {
        CHECK(serve_cancel(s, a) == VECCHIA_OK);      // cancelled while queued ...
        waiting = a;
    }
    CHECK(serve_release(s, waiting) == VECCHIA_OK);   // ... and freed at once
    // a large request whose graph is still being built when it is cancelled
    std::vector<double> big = points(90000, 3, 9);
    CHECK(serve_submit(s, big.data(), 90000, 8, 128, &kern, VECCHIA_OP_LOGDET, nullptr, &c) == VECCHIA_OK);
    const int rc_cancel = serve_cancel(s, c);
    CHECK(rc_cancel == VECCHIA_OK);
    while (serve_release(s, c) != VECCHIA_OK) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    // more traffic through the same queues after the frees
    std::vector<int64_t> ids;
    for (int i = 0; i < 6; ++i) {
        int64_t id = 0;
        std::vector<double> xi = points(1000 + 500 * i, 3, 100 + i);
        std::vector<float> vi(xi.size() / 3, (float)i);
        CHECK(serve_submit(s, xi.data(), (int64_t)vi.size(), 8, 64, &kern, VECCHIA_OP_FORWARD, vi.data(), &id) ==
              VECCHIA_OK);
        ids.push_back(id);
    }
    int finished = 0;
    for (int it = 0; it < 200000 && finished < 7; ++it) {
        CHECK(serve_progress(s, &done) == VECCHIA_OK);
        int64_t id = 0;
        while (serve_take(s, &id) == VECCHIA_OK && id) {
            double t[4];
            std::vector<float> out(60000);
            CHECK(serve_result(s, id, out.data(), nullptr, t) == VECCHIA_OK);
            CHECK(serve_release(s, id) == VECCHIA_OK);
            ++finished;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    CHECK(finished == 7);
    vecchia_serve_stats st;
    CHECK(serve_stats(s, &st) == VECCHIA_OK);
    CHECK(st.bytes_in_use == 0 && st.cancelled == 2 && st.completed == 7);
    serve_destroy(s);
}

int main() {
    graphs();
    scheduler();
    std::printf("host driver ok\n");
    return 0;
}
