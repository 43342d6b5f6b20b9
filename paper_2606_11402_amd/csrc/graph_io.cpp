// Graph files (graph_save / graph_load, declared in vecchia.h with their
// layout).  Loading rebuilds the graph from the stored points, tree, rows and
// depths through the checked entry points of the device build
// (graph_build_begin_tree, graph_build_finish_depth), so a file can only
// yield a graph that passes the same checks as one built here.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "graph_internal.h"
#include "status.h"
#include "vecchia.h"

namespace {

constexpr char kGraphMagic[8] = {'V', 'C', 'G', 'R', 'A', 'P', 'H', '1'};

struct Fnv1a {
    uint64_t h = 0xcbf29ce484222325ull;   // FNV-1a 64-bit offset basis
    void add(const void* p, size_t n) {
        const unsigned char* c = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;   // FNV 64-bit prime
    }
};

struct FileCloser {
    FILE* f;
    ~FileCloser() {
        if (f) fclose(f);
    }
};

bool write_part(FILE* f, Fnv1a& h, const void* p, size_t n) {
    h.add(p, n);
    return n == 0 || fwrite(p, 1, n, f) == n;
}

bool read_part(FILE* f, Fnv1a& h, void* p, size_t n) {
    if (n != 0 && fread(p, 1, n, f) != n) return false;
    h.add(p, n);
    return true;
}

}  // namespace

extern "C" int graph_save(const vecchia_graph* g, const char* path) {
    vecchia_clear_error();
    if (!g || !path) return vecchia_set_error(VECCHIA_EINVAL, "graph_save: NULL argument");
    if (g->pending) return vecchia_set_error(VECCHIA_EINVAL, "graph_save: graph is pending (build not finished)");
    const int64_t n = g->n, ns = g->n - g->n0;
    const int d = g->d, k = g->k;
    std::vector<double> x;
    std::vector<int32_t> sdim, rows;
    try {
        x.resize((size_t)n * d);
        sdim.resize(n);
        rows.resize((size_t)ns * k);
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = g->tree_perm[t];
            for (int c = 0; c < d; ++c) x[i * d + c] = g->xs[t * 3 + c];
            sdim[t] = g->sdim[t];
        }
        // stored rows are in-order ranks; the file holds slot numbers
        for (size_t q = 0; q < rows.size(); ++q) rows[q] = g->nbr[q] >= 0 ? g->seq[g->nbr[q]] : -1;
    } catch (const std::bad_alloc&) {
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_save: host allocation failed");
    }
    FileCloser fc{fopen(path, "wb")};
    if (!fc.f) return vecchia_set_error(VECCHIA_EIO, "graph_save: cannot open %s for writing", path);
    Fnv1a h;
    const int32_t hdr32[4] = {d, k, g->n0, 0};
    bool ok = write_part(fc.f, h, kGraphMagic, 8) && write_part(fc.f, h, &n, 8) && write_part(fc.f, h, hdr32, 16) &&
              write_part(fc.f, h, x.data(), x.size() * sizeof(double)) &&
              write_part(fc.f, h, g->tree_perm.data(), (size_t)n * 4) && write_part(fc.f, h, sdim.data(), (size_t)n * 4) &&
              write_part(fc.f, h, rows.data(), rows.size() * 4) && write_part(fc.f, h, g->depth.data(), (size_t)n * 4);
    const uint64_t digest = h.h;
    ok = ok && fwrite(&digest, 1, 8, fc.f) == 8;
    const bool closed = fclose(fc.f) == 0;
    fc.f = nullptr;
    if (!ok || !closed) return vecchia_set_error(VECCHIA_EIO, "graph_save: writing %s failed", path);
    return VECCHIA_OK;
}

extern "C" int graph_load(const char* path, int32_t n_threads, vecchia_graph** out) {
    vecchia_clear_error();
    if (!path || !out) return vecchia_set_error(VECCHIA_EINVAL, "graph_load: NULL argument");
    *out = nullptr;
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) return vecchia_set_error(VECCHIA_EIO, "graph_load: cannot open %s", path);
    Fnv1a h;
    char magic[8];
    int64_t n = 0;
    int32_t hdr32[4];
    if (!read_part(fc.f, h, magic, 8) || std::memcmp(magic, kGraphMagic, 8) != 0)
        return vecchia_set_error(VECCHIA_EIO, "graph_load: %s is not a graph file", path);
    if (!read_part(fc.f, h, &n, 8) || !read_part(fc.f, h, hdr32, 16))
        return vecchia_set_error(VECCHIA_EIO, "graph_load: %s is truncated (header)", path);
    const int32_t d = hdr32[0], k = hdr32[1], n0 = hdr32[2];
    // the sizes bound the allocations below; the build arguments proper are
    // checked again by graph_build_begin_tree
    if (n < 1 || n >= (int64_t(1) << 31) || d < 1 || d > 3 || k < 1 || n0 < 1 || n0 > n || hdr32[3] != 0)
        return vecchia_set_error(VECCHIA_EIO, "graph_load: %s has an invalid header", path);
    if (k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "graph_load: k=%d exceeds the compiled maximum %d", k, VECCHIA_KMAX);
    // the file's length must be the one its header implies, checked before
    // anything of that size is allocated
    const int64_t want = 32 + n * d * 8 + 4 * (3 * n + (n - n0) * (int64_t)k) + 8;
    const long here = ftell(fc.f);
    if (here < 0 || fseek(fc.f, 0, SEEK_END) != 0)
        return vecchia_set_error(VECCHIA_EIO, "graph_load: cannot seek in %s", path);
    const long len = ftell(fc.f);
    if (len < 0 || fseek(fc.f, here, SEEK_SET) != 0)
        return vecchia_set_error(VECCHIA_EIO, "graph_load: cannot seek in %s", path);
    if ((int64_t)len != want)
        return vecchia_set_error(VECCHIA_EIO, "graph_load: %s has %lld bytes, its header implies %lld", path,
                                 (long long)len, (long long)want);
    std::vector<double> x;
    std::vector<int32_t> perm, sdim, rows, depth;
    try {
        x.resize((size_t)n * d);
        perm.resize(n);
        sdim.resize(n);
        rows.resize((size_t)(n - n0) * k);
        depth.resize(n);
    } catch (const std::bad_alloc&) {
        return vecchia_set_error(VECCHIA_ENOMEM, "graph_load: host allocation failed (N=%lld)", (long long)n);
    }
    uint64_t digest = 0;
    if (!read_part(fc.f, h, x.data(), x.size() * sizeof(double)) || !read_part(fc.f, h, perm.data(), (size_t)n * 4) ||
        !read_part(fc.f, h, sdim.data(), (size_t)n * 4) || !read_part(fc.f, h, rows.data(), rows.size() * 4) ||
        !read_part(fc.f, h, depth.data(), (size_t)n * 4) || fread(&digest, 1, 8, fc.f) != 8)
        return vecchia_set_error(VECCHIA_EIO, "graph_load: %s is truncated", path);
    char extra;
    if (fread(&extra, 1, 1, fc.f) != 0) return vecchia_set_error(VECCHIA_EIO, "graph_load: %s has trailing bytes", path);
    if (digest != h.h) return vecchia_set_error(VECCHIA_EIO, "graph_load: %s fails its hash (damaged file)", path);
    vecchia_graph* g = nullptr;
    int rc = graph_build_begin_tree(x.data(), n, d, k, n0, n_threads, perm.data(), sdim.data(), &g);
    if (rc) return rc;
    const int32_t no_rows = -1;   // N == n0: no sparse rows, but the pointer must not be NULL
    rc = graph_build_finish_depth(g, rows.empty() ? &no_rows : rows.data(), depth.data());
    if (rc) {
        graph_free(g);
        return rc;
    }
    *out = g;
    return VECCHIA_OK;
}
