// The host graph object shared by the builder (graph.cpp) and the graph
// files (graph_io.cpp).  Not part of the C ABI: callers hold a
// vecchia_graph* and use the graph_* calls of vecchia.h.
#pragma once

#include <cstdint>
#include <vector>

#include "vecchia.h"

struct vecchia_graph {
    int64_t n = 0;
    int32_t d = 0, k = 0, kp = 0, n0 = 0, n_levels = 0;
    std::vector<double> xs;            // slot order, 3 per slot (zero padded)
    std::vector<int32_t> tree_perm;    // slot -> input index
    std::vector<int8_t> sdim;          // slot -> split dimension
    std::vector<int32_t> nbr;          // (n - n0) x k neighbours as in-order ranks, row r = slot n0 + r
    std::vector<int32_t> seq;          // in-order rank -> slot
    std::vector<int32_t> rank_of;      // slot -> in-order rank
    std::vector<int32_t> depth;        // slot -> depth
    std::vector<int32_t> order;        // storage -> slot
    std::vector<int32_t> pos;          // slot -> storage
    std::vector<int32_t> pos_r;        // in-order rank -> storage
    std::vector<int32_t> level_ptr;    // n_levels + 2
    int nthreads = 1;                  // host threads of the build, reused by the exports
    double times[4] = {0, 0, 0, 0};
    bool pending = false;              // begun (tree only): neighbours, depths and storage still missing
};
