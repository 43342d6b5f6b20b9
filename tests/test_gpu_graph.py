"""The k-d tree on the device (graph_tree_device), the preceding k-NN search
on the device (graph_knn_device) and the depth fixpoint on the device
(graph_depth_device) give the same graph as the host builder, bit for bit (the host builder is itself bit-exact with the oracle's
brute-force search and depth recurrence, tests/test_graph_native.py): same
order, same depths and batches, same neighbour rows in both layouts."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2606_11402_amd import Graph

pytestmark = pytest.mark.gpu


def same_graph(a, b):
    assert (a.order == b.order).all() and (a.slot == b.slot).all()
    assert (a.depth == b.depth).all() and (a.level_ptr == b.level_ptr).all()
    assert (a.nbr(0) == b.nbr(0)).all() and (a.nbr(1) == b.nbr(1)).all()


@pytest.mark.parametrize("n,d,k,n0,seed", [
    (3000, 3, 8, 32, 0), (2000, 2, 16, 16, 1), (1500, 1, 5, 3, 2), (4000, 3, 32, 32, 3),
    (777, 3, 32, 1, 4), (1500, 3, 64, 64, 12), (300, 3, 64, 1, 13), (65, 3, 8, 64, 6),
])
def test_device_knn_equals_host(n, d, k, n0, seed):
    x = np.random.default_rng(seed).random((n, d))
    same_graph(Graph(x, k, n0, knn_device="cuda:0"), Graph(x, k, n0))


def test_device_knn_ties_and_duplicates():
    grid = np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    same_graph(Graph(grid, 8, 8, knn_device="cuda:0"), Graph(grid, 8, 8))
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1500, 3)) * (10.0 ** rng.uniform(-3, 0, 1500))[:, None]
    x[100:120] = x[5]
    g = Graph(x, 16, 16, knn_device="cuda:0")
    same_graph(g, Graph(x, 16, 16))
    og = oracle.build_graph(x, 16, 16)                   # and directly against brute force
    nb = g.nbr(0)
    mapped = np.where(nb >= 0, g.slot[np.maximum(nb, 0)], -1)
    assert (mapped == og.nbr[g.slot[16:] - 16]).all()


def test_device_knn_workload3_distribution_2e20():
    w = workloads.WORKLOADS[3]
    x = w.points(1 << 20)
    g = Graph(x, 32, 128, knn_device="cuda:0")
    print("device knn seconds (incl. transfers)", g.knn_seconds, "depth sweeps", g.depth_sweeps,
          g.split_seconds, flush=True)
    assert g.depth_sweeps is not None and g.depth_sweeps >= 1
    same_graph(g, Graph(x, 32, 128))


@pytest.mark.parametrize("wl,n,k", [(2, 1 << 18, 16), (1, 50000, 8), (3, 1 << 18, 64)])
def test_device_depth_with_and_without(wl, n, k):
    """The depth fixpoint on the device against the host's depth pass after
    the same device neighbour search, and against the host build."""
    w = workloads.WORKLOADS[wl]
    x = w.points(n)
    a = Graph(x, k, 32, knn_device="cuda:0", depth_device=True)
    b = Graph(x, k, 32, knn_device="cuda:0", depth_device=False)
    print("workload", wl, "n", n, "k", k, "levels", a.n_levels, "sweeps", a.depth_sweeps, flush=True)
    assert a.depth_sweeps is not None and b.depth_sweeps is None
    same_graph(a, b)
    same_graph(a, Graph(x, k, 32))


def test_device_tree_signed_zeros_and_ties():
    """Coordinates that tie, including -0.0 against +0.0 (equal for the
    tree's key), on a small integer grid centred on zero."""
    g1 = np.stack(np.meshgrid(*[np.arange(-3, 4)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    neg = np.random.default_rng(3).random(g1.shape) < 0.5
    g1[(g1 == 0) & neg] = -0.0
    assert np.signbit(g1[g1 == 0]).any() and (~np.signbit(g1[g1 == 0])).any()
    for k, n0 in ((8, 8), (16, 1)):
        a = Graph(g1, k, n0, knn_device="cuda:0")
        print("signed zeros: tree seconds", a.tree_seconds, flush=True)
        same_graph(a, Graph(g1, k, n0))


@pytest.mark.parametrize("tree,depth", [(True, False), (False, True)])
def test_device_steps_one_at_a_time(tree, depth):
    w = workloads.WORKLOADS[2]
    x = w.points(1 << 17)
    a = Graph(x, 16, 64, knn_device="cuda:0", tree_device=tree, depth_device=depth)
    same_graph(a, Graph(x, 16, 64))
