"""Pins of the preceding-neighbour graph and the depth batches."""
import json
import os

import numpy as np
import pytest
import scipy.spatial

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_1d_graph_with_ties():
    g = json.load(open(os.path.join(GOLDEN, "graph_1d_n10.json")))
    xs = np.asarray(g["xs_1d"], dtype=np.float64)[:, None]
    nbr = oracle.preceding_knn(xs, g["k"], g["n0"])
    assert nbr.tolist() == g["nbr_rows_for_slots_2_to_9"]
    d = oracle.depths(nbr, len(xs), g["n0"])
    assert d.tolist() == g["depth"]
    for lev, slots in g["levels"].items():
        assert np.nonzero(d == int(lev))[0].tolist() == slots


def test_golden_graph_through_tree():
    # the tree of tree_1d_n10.json feeds the graph of graph_1d_n10.json
    t = json.load(open(os.path.join(GOLDEN, "tree_1d_n10.json")))
    g = json.load(open(os.path.join(GOLDEN, "graph_1d_n10.json")))
    gr = oracle.build_graph(np.asarray(t["points_1d"], dtype=np.float64), g["k"], g["n0"])
    assert gr.nbr.tolist() == g["nbr_rows_for_slots_2_to_9"]
    assert gr.depth.tolist() == g["depth"]


@pytest.mark.parametrize("n,k,n0,seed", [(600, 8, 16, 0), (400, 16, 16, 1), (300, 5, 2, 2)])
def test_knn_against_ckdtree(n, k, n0, seed):
    xs = np.random.default_rng(seed).random((n, 3))
    nbr = oracle.preceding_knn(xs, k, n0)
    for i in range(n0, n):
        m = min(k, i)
        tree = scipy.spatial.cKDTree(xs[:i])
        q = min(m + 1, i)
        dist, idx = tree.query(xs[i], k=q)
        dist, idx = np.atleast_1d(dist), np.atleast_1d(idx)
        row = nbr[i - n0]
        assert (row[m:] == -1).all()
        ours = np.sqrt(np.sum((xs[row[:m]] - xs[i]) ** 2, axis=1))
        np.testing.assert_allclose(ours, dist[:m], rtol=1e-12)
        if q == m or dist[m] > dist[m - 1] * (1 + 1e-9):      # no near-tie at the cut
            assert set(row[:m].tolist()) == set(idx[:m].tolist())


@pytest.mark.parametrize("seed", [0, 1])
def test_depth_invariants(seed):
    n, k, n0 = 800, 8, 32
    gr = oracle.build_graph(np.random.default_rng(seed).random((n, 3)), k, n0)
    assert (gr.depth[:n0] == 0).all()
    for i in range(n0, n):
        row = gr.nbr[i - n0]
        row = row[row >= 0]
        assert (row < i).all() and len(set(row.tolist())) == len(row)
        assert (gr.depth[row] < gr.depth[i]).all()
        assert (gr.depth[row] == gr.depth[i] - 1).any()
    # levels partition the sparse slots, and no slot depends on its own level
    all_lv = np.concatenate([gr.level_slots(l) for l in range(1, gr.n_levels + 1)])
    assert sorted(all_lv.tolist()) == list(range(n0, n))
    so = gr.order
    assert (np.diff(gr.depth[so]) >= 0).all() and so[:n0].tolist() == list(range(n0))


def test_bit_reversed_batches_are_large():
    """Sec. 2.2: the bit-reversed order yields few, large batches.  (The
    figure with the paper's batch sizes is absent: counts are unpinned; this
    only checks that the number of batches grows much slower than N.)"""
    x = np.random.default_rng(7).standard_normal((4000, 3))
    gr = oracle.build_graph(x, 16, 50)
    assert gr.n_levels < 200
