"""The C++ graph build (host, int32) against the oracle, bit for bit."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2606_11402_amd import _lib
from paper_2606_11402_amd import Graph, VecchiaError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def compare(x, k, n0, rows=None):
    g = Graph(x, k, n0)
    og = oracle.build_graph(x, k, n0) if rows is None else None
    return g, og


def assert_same_graph(g, og):
    n0 = g.n0
    assert (og.perm[g.slot] == g.order).all()
    nb = g.nbr(0)
    mapped = np.where(nb >= 0, g.slot[np.maximum(nb, 0)], -1)
    assert (mapped == og.nbr[g.slot[n0:] - n0]).all()
    assert (g.depth == og.depth[g.slot]).all()
    assert g.n_levels == og.n_levels
    assert g.slot[:n0].tolist() == list(range(n0))
    for lev in range(1, g.n_levels + 1):
        a, b = g.level_ptr[lev], g.level_ptr[lev + 1]
        assert sorted(g.slot[a:b].tolist()) == og.level_slots(lev).tolist()


def test_golden_1d():
    t = json.load(open(os.path.join(GOLDEN, "tree_1d_n10.json")))
    gj = json.load(open(os.path.join(GOLDEN, "graph_1d_n10.json")))
    g = Graph(np.asarray(t["points_1d"], dtype=np.float64), gj["k"], gj["n0"])
    assert g.order[np.argsort(g.slot)].tolist() == t["perm"]
    nb = g.nbr(0)
    rows = {int(g.slot[g.n0 + r]): [int(g.slot[j]) for j in nb[r]] for r in range(g.ns)}
    assert [rows[s] for s in range(2, 10)] == gj["nbr_rows_for_slots_2_to_9"]


@pytest.mark.parametrize("n,d,k,n0,seed", [
    (3000, 3, 8, 32, 0), (2000, 2, 16, 16, 1), (1500, 1, 5, 3, 2), (4000, 3, 32, 32, 3),
    (777, 3, 32, 1, 4),        # padded rows: n0 < k
    (64, 3, 8, 64, 5),         # dense block only
    (65, 3, 8, 64, 6),         # one sparse point
    (1500, 3, 64, 64, 12),     # the widest compiled neighbour count
    (300, 3, 64, 1, 13),       # k = 64 with padded rows
])
def test_bit_exact_against_oracle(n, d, k, n0, seed):
    x = np.random.default_rng(seed).random((n, d))
    g = Graph(x, k, n0)
    assert_same_graph(g, oracle.build_graph(x, k, n0))


def test_ties_integer_grid():
    x = np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    g = Graph(x, 8, 8)
    assert_same_graph(g, oracle.build_graph(x, 8, 8))


def test_duplicates_and_dynamic_range():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1500, 3)) * (10.0 ** rng.uniform(-3, 0, 1500))[:, None]
    x[100:120] = x[5]
    g = Graph(x, 16, 16)
    assert_same_graph(g, oracle.build_graph(x, 16, 16))


@pytest.mark.slow
def test_sampled_rows_large():
    """N = 2^16 radial cloud: the whole tree order and sampled neighbour rows
    (first and last 512 rows plus 2048 random) against brute force."""
    import workloads
    x = workloads.as_fp32_exact(workloads.radial(1 << 16, 2))
    k, n0 = 16, 128
    g = Graph(x, k, n0)
    perm, _ = oracle.tree_order(x)
    assert (perm[g.slot] == g.order).all()
    xs = x[perm]
    nb = g.nbr(0)
    pos = np.empty(g.n, np.int64)
    pos[g.slot] = np.arange(g.n)
    rng = np.random.default_rng(11)
    slots = np.unique(np.concatenate([np.arange(n0, n0 + 512), np.arange(g.n - 512, g.n),
                                      rng.integers(n0, g.n, 2048)]))
    for s in slots:
        ref = oracle.preceding_knn(xs[:s + 1], k, s)[0]
        got = g.slot[nb[pos[s] - n0]]
        assert (got == ref).all()


def test_tiled_layout_matches_row_major():
    x = np.random.default_rng(8).random((1000, 3))
    g = Graph(x, 12, 41)                  # Ns = 959: ragged last tile
    rm = g.nbr(0)
    tl = g.nbr(1).reshape(g.ntiles, g.kp, 64)
    for sp in (0, 1, 63, 64, 500, g.ns - 1):
        row = tl[sp // 64, :, sp % 64]
        # the device row holds the same neighbours, ascending storage position
        assert row[:12].tolist() == sorted(rm[sp].tolist()) and (row[12:] == -1).all()
    assert (tl.reshape(g.ntiles, g.kp, 64)[-1, :, g.ns % 64:] == -1).all()


@pytest.mark.parametrize("n,k,n_threads", [(150001, 16, 8), (70000, 32, 3)])
def test_children_lists_against_the_device_rows(n, k, n_threads):
    """Children lists of a cloud large enough for the threaded export, against
    the inversion of the device rows written out with NumPy: list j holds the
    packed entries sp * kp + m with row sp naming j at position m, ascending."""
    x = np.random.default_rng(n).random((n, 3))
    g = Graph(x, k, 64, n_threads=n_threads)
    ptr, child = g.children()
    nb = g.nbr(1).reshape(g.ntiles, g.kp, 64).transpose(0, 2, 1).reshape(-1, g.kp)[:g.ns]
    sp, m = np.nonzero(nb >= 0)
    j = nb[sp, m].astype(np.int64)
    entry = sp.astype(np.int64) * g.kp + m
    key = np.lexsort((entry, j))
    want_ptr = np.concatenate([[0], np.cumsum(np.bincount(j, minlength=g.n))])
    assert (ptr == want_ptr).all()
    assert (child[:ptr[-1]] == entry[key]).all()


def test_children_lists_invert_neighbours():
    x = np.random.default_rng(9).random((800, 3))
    g = Graph(x, 8, 16)
    ptr, child = g.children()
    nb = g.nbr(1).reshape(g.ntiles, g.kp, 64).transpose(0, 2, 1).reshape(-1, g.kp)[:g.ns]   # device rows
    seen = np.zeros_like(nb, dtype=bool)
    for j in range(g.n):
        entries = child[ptr[j]:ptr[j + 1]]
        assert (np.diff(entries) > 0).all()
        for e in entries:
            sp, m = divmod(int(e), g.kp)
            assert nb[sp, m] == j
            seen[sp, m] = True
    assert seen[nb >= 0].all()


@pytest.mark.parametrize("args", [
    dict(k=0, n0=4, code=-1), dict(k=_lib.KMAX + 1, n0=40, code=-4), dict(k=4, n0=0, code=-1),
    dict(k=4, n0=2000, code=-1),
])
def test_invalid_arguments(args):
    """Invalid arguments are EINVAL (-1); a neighbour count above the compiled
    maximum is EUNSUPPORTED (-4)."""
    x = np.random.default_rng(0).random((100, 3))
    with pytest.raises(VecchiaError) as e:
        Graph(x, args["k"], args["n0"])
    assert e.value.code == args["code"]


def test_non_finite_rejected():
    x = np.random.default_rng(0).random((100, 3))
    x[50, 1] = np.nan
    with pytest.raises(VecchiaError):
        Graph(x, 4, 8)


def test_storage_order_is_spatially_coherent_inside_levels():
    """Inside a batch, points follow the tree's in-order sequence: consecutive
    storage positions are much closer than random pairs."""
    x = np.random.default_rng(10).random((20000, 3))
    g = Graph(x, 8, 64)
    xs = g.points()
    a, b = g.level_ptr[g.n_levels // 2], g.level_ptr[g.n_levels // 2 + 1]
    if b - a > 100:
        consecutive = np.linalg.norm(np.diff(xs[a:b], axis=0), axis=1).mean()
        rnd = np.linalg.norm(xs[a:b] - xs[np.random.default_rng(0).permutation(np.arange(a, b))], axis=1).mean()
        assert consecutive < 0.5 * rnd


def test_row_order_helper_inverts_the_device_order():
    # Graph.to_row_order maps values laid out along the device rows back to
    # the rows of nbr(0); applied to the device rows' own indices it must
    # give nbr(0) exactly (padded rows included)
    for n, k, n0 in ((1000, 12, 41), (300, 32, 5)):
        x = np.random.default_rng(n).random((n, 3))
        g = Graph(x, k, n0)
        dev = g.nbr(1).reshape(g.ntiles, g.kp, 64).transpose(0, 2, 1).reshape(-1, g.kp)[:g.ns]
        back = g.to_row_order(dev.astype(np.int64))
        rm = g.nbr(0)
        pad = rm < 0
        assert (back[~pad] == rm[~pad]).all() and (back[pad] == -1).all()
        rows = np.array([0, 7, g.ns - 1])
        assert (g.to_row_order(dev[rows].astype(np.int64), rows)[~pad[rows]] == rm[rows][~pad[rows]]).all()


def _begin(x, k, n0):
    lib = _lib.load()
    import ctypes
    x = np.ascontiguousarray(x, dtype=np.float64)
    h = ctypes.c_void_p()
    _lib.check(lib.graph_build_begin(x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), x.shape[0], x.shape[1], k,
                                     n0, 2, ctypes.byref(h)), "graph_build_begin")
    return lib, h


@pytest.mark.parametrize("n,d,k,n0,seed", [(1500, 3, 8, 32, 40), (900, 2, 16, 4, 41), (300, 3, 64, 1, 42)])
def test_split_build_with_brute_force_rows_equals_graph_build(n, d, k, n0, seed):
    """graph_build_begin + graph_build_finish fed the oracle's brute-force
    rows (tree slots, ascending (D, slot), -1 padded) gives exactly the graph
    of graph_build: the order, the batches and every exported row."""
    import ctypes
    x = np.random.default_rng(seed).random((n, d))
    og = oracle.build_graph(x, k, n0)
    lib, h = _begin(x, k, n0)
    rows = np.ascontiguousarray(og.nbr.astype(np.int32))
    assert lib.graph_export_nbr(h, 0, ctypes.c_void_p(np.empty(1, np.int32).ctypes.data)) == _lib.EINVAL  # pending
    _lib.check(lib.graph_build_finish(h, ctypes.c_void_p(rows.ctypes.data)), "graph_build_finish")
    ref = Graph(x, k, n0)
    got_order = np.empty(n, np.int32)
    got_lp = np.empty(ref.n_levels + 2, np.int32)
    _lib.check(lib.graph_export(h, ctypes.c_void_p(got_order.ctypes.data), None, ctypes.c_void_p(got_lp.ctypes.data),
                                None), "graph_export")
    assert (got_order == ref.order).all() and (got_lp == ref.level_ptr).all()
    for layout in (0, 1):
        size = (n - n0) * k if layout == 0 else ref.ntiles * ref.kp * 64
        got = np.empty(max(size, 1), np.int32)
        _lib.check(lib.graph_export_nbr(h, layout, ctypes.c_void_p(got.ctypes.data)), "graph_export_nbr")
        assert (got[:size] == ref.nbr(layout).reshape(-1)).all()
    lib.graph_free(h)


def test_split_build_rejects_bad_rows():
    import ctypes
    x = np.random.default_rng(5).random((400, 3))
    og = oracle.build_graph(x, 8, 16)
    for mutate in ("later_slot", "order", "missing"):
        rows = np.ascontiguousarray(og.nbr.astype(np.int32))
        if mutate == "later_slot":
            rows[100, 0] = 16 + 100           # its own slot: not a predecessor
        elif mutate == "order":
            rows[200, [0, 1]] = rows[200, [1, 0]]
        else:
            rows[300, 3] = -1                 # padding inside a full row
        lib, h = _begin(x, 8, 16)
        assert lib.graph_build_finish(h, ctypes.c_void_p(rows.ctypes.data)) == _lib.EINVAL, mutate
        lib.graph_free(h)


def _slot_depths(g):
    d = np.empty(g.n, np.int32)
    d[g.slot] = g.depth
    return d


def test_split_build_with_given_depths_equals_graph_build():
    """graph_build_finish_depth fed the brute-force rows and the host
    builder's depths (tree slot order) gives the graph of graph_build; a depth
    that breaks the recurrence is EINVAL."""
    import ctypes
    x = np.random.default_rng(21).random((1200, 3))
    k, n0 = 8, 16
    og = oracle.build_graph(x, k, n0)
    ref = Graph(x, k, n0)
    rows = np.ascontiguousarray(og.nbr.astype(np.int32))
    depth = _slot_depths(ref)
    lib, h = _begin(x, k, n0)
    _lib.check(lib.graph_build_finish_depth(h, ctypes.c_void_p(rows.ctypes.data), ctypes.c_void_p(depth.ctypes.data)),
               "graph_build_finish_depth")
    got_order = np.empty(1200, np.int32)
    got_lp = np.empty(ref.n_levels + 2, np.int32)
    _lib.check(lib.graph_export(h, ctypes.c_void_p(got_order.ctypes.data), None, ctypes.c_void_p(got_lp.ctypes.data),
                                None), "graph_export")
    assert (got_order == ref.order).all() and (got_lp == ref.level_ptr).all()
    lib.graph_free(h)
    for i, delta in ((700, 1), (300, -1), (3, 1)):          # a sparse slot one too deep or shallow; a dense one
        bad = depth.copy()
        bad[i] += delta
        lib, h = _begin(x, k, n0)
        assert lib.graph_build_finish_depth(h, ctypes.c_void_p(rows.ctypes.data), ctypes.c_void_p(bad.ctypes.data)) \
            == _lib.EINVAL
        lib.graph_free(h)


@pytest.mark.parametrize("n,d,seed", [(1500, 3, 30), (700, 2, 31), (300, 1, 32), (1, 3, 33), (2, 2, 34)])
def test_begin_from_given_tree_equals_graph_build(n, d, seed):
    """graph_build_begin_tree fed the oracle's tree (Sec. 2.2) and then the
    brute-force rows gives the graph of graph_build."""
    import ctypes
    x = np.random.default_rng(seed).random((n, d))
    k, n0 = 8, 1
    perm, sdim = oracle.tree_order(x)
    perm, sdim = np.ascontiguousarray(perm.astype(np.int32)), np.ascontiguousarray(sdim.astype(np.int32))
    lib = _lib.load()
    h = ctypes.c_void_p()
    xc = np.ascontiguousarray(x)
    _lib.check(lib.graph_build_begin_tree(xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, d, k, n0, 2,
                                          ctypes.c_void_p(perm.ctypes.data), ctypes.c_void_p(sdim.ctypes.data),
                                          ctypes.byref(h)), "graph_build_begin_tree")
    og = oracle.build_graph(x, k, n0)
    rows = np.ascontiguousarray(og.nbr.astype(np.int32)) if n > n0 else np.zeros(1, np.int32)
    _lib.check(lib.graph_build_finish(h, ctypes.c_void_p(rows.ctypes.data)), "graph_build_finish")
    ref = Graph(x, k, n0)
    got = np.empty(n, np.int32)
    _lib.check(lib.graph_export(h, ctypes.c_void_p(got.ctypes.data), None, None, None), "graph_export")
    assert (got == ref.order).all()
    lib.graph_free(h)


def test_begin_from_given_tree_rejects_other_trees():
    """A tree that is not the one of the points is EINVAL: two slots swapped,
    a split dimension changed, an index repeated."""
    import ctypes
    rng = np.random.default_rng(35)
    x = rng.random((900, 3)) * np.array([1.0, 0.5, 0.25])
    perm, sdim = oracle.tree_order(x)
    lib = _lib.load()
    xc = np.ascontiguousarray(x)
    xp = xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cases = []
    p = perm.copy(); p[[5, 600]] = p[[600, 5]]; cases.append((p, sdim))
    s = sdim.copy(); s[0] = (s[0] + 1) % 3; cases.append((perm, s))
    s = sdim.copy(); s[400] = 2 if s[400] != 2 else 1; cases.append((perm, s))
    p = perm.copy(); p[10] = p[11]; cases.append((p, sdim))
    p = perm.copy(); p[1], p[2] = p[2], p[1]; cases.append((p, sdim))
    for p, s in cases:
        p = np.ascontiguousarray(p.astype(np.int32))
        s = np.ascontiguousarray(s.astype(np.int32))
        h = ctypes.c_void_p()
        assert lib.graph_build_begin_tree(xp, 900, 3, 8, 16, 2, ctypes.c_void_p(p.ctypes.data),
                                          ctypes.c_void_p(s.ctypes.data), ctypes.byref(h)) == _lib.EINVAL


def test_thread_count_does_not_change_the_graph():
    """The threaded phases (neighbour search, depths, the chunked counting
    sort of the storage order) give the graph of the one-thread build."""
    x = np.random.default_rng(21).random((150001, 3))
    g1 = Graph(x, 8, 64, n_threads=1)
    g4 = Graph(x, 8, 64, n_threads=4)
    for name in ("order", "slot", "depth", "level_ptr"):
        assert (getattr(g1, name) == getattr(g4, name)).all(), name
    assert (g1.nbr(1) == g4.nbr(1)).all()
    p1, c1 = g1.children()
    p4, c4 = g4.children()
    assert (p1 == p4).all() and (c1 == c4).all()


@pytest.mark.parametrize("n,n_threads", [(1000, 1), (70001, 4), (262147, 8)])
def test_batches_follow_the_in_order_sequence(n, n_threads):
    """In one dimension the tree is a binary search tree on (coordinate,
    input index), so its in-order sequence is the sorted order: inside every
    batch the storage order must ascend by that key (Sec. 2.2, batch
    construction; the in-order layout inside a batch)."""
    rng = np.random.default_rng(n)
    x = np.round(rng.random(n), 3)                 # many ties
    g = Graph(x, 4, 32, n_threads=n_threads)
    for lev in range(1, g.n_levels + 1):
        a, b = g.level_ptr[lev], g.level_ptr[lev + 1]
        idx = g.order[a:b].astype(np.int64)
        key = np.lexsort((idx, x[idx]))
        assert (key == np.arange(b - a)).all(), lev
