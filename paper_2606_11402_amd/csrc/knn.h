// Node of the query tree of the preceding k-NN search (Sec. 2.1), shared by
// the host builder (graph.cpp) and the device search (knn.hip): the tree of
// the bit-reversed order laid out in in-order sequence, so that every
// subtree occupies one contiguous range of ranks.
#pragma once

#include <cstdint>

struct KnnNode {
    double c[3];            // coordinates (zero padded for d < 3)
    int32_t slot;           // tree slot of the node's point
    int32_t left, right;    // in-order ranks of the children, -1 if absent
    int32_t sdim;           // split dimension
};
static_assert(sizeof(KnnNode) == 40, "KnnNode layout");
