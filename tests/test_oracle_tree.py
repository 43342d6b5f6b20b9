"""Pins of the bit-reversed k-d tree order (Sec. 2.2)."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_1d_n10():
    g = json.load(open(os.path.join(GOLDEN, "tree_1d_n10.json")))
    perm, _ = oracle.tree_order(np.asarray(g["points_1d"], dtype=np.float64))
    assert perm.tolist() == g["perm"]


def heap_median_tree(x):
    """Plain heap-order (children 2h+1, 2h+2) median k-d tree, written here
    independently of the oracle; same split rule and tie order."""
    n = len(x)
    out = np.full(n, -1)

    def rec(h, subset):
        if len(subset) == 0:
            return
        ext = x[subset].max(0) - x[subset].min(0)
        s = int(np.argmax(ext))
        subset = sorted(subset, key=lambda i: (x[i, s], i))
        m = len(subset) // 2
        out[h] = subset[m]
        rec(2 * h + 1, subset[:m])
        rec(2 * h + 2, subset[m + 1:])

    rec(0, list(range(n)))
    return out


def bitrev(q, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (q & 1)
        q >>= 1
    return r


@pytest.mark.parametrize("levels", [1, 2, 3, 5, 8])
def test_full_tree_is_levelwise_bit_reversal_of_heap_order(levels):
    n = (1 << levels) - 1
    x = np.random.default_rng(levels).random((n, 3))
    heap = heap_median_tree(x)
    perm, _ = oracle.tree_order(x)
    for l in range(levels):
        for q in range(1 << l):
            slot = (1 << l) - 1 + q
            heap_pos = (1 << l) - 1 + bitrev(q, l)
            assert perm[slot] == heap[heap_pos]


def subtree(t, n):
    out, stack = [], [t]
    while stack:
        u = stack.pop()
        if u < n:
            out.append(u)
            stack += [oracle.left_child(u), oracle.right_child(u)]
    return out


@pytest.mark.parametrize("n,seed", [(10, 0), (37, 1), (200, 2), (1000, 3)])
def test_invariants_ragged(n, seed):
    x = np.random.default_rng(seed).random((n, 3))
    x[:, 2] *= 0.1                                  # anisotropic: exercises the split rule
    perm, sdim = oracle.tree_order(x)
    assert sorted(perm.tolist()) == list(range(n))
    for t in range(n):
        l, r = oracle.left_child(t), oracle.right_child(t)
        ls, rs = subtree(l, n), subtree(r, n)
        assert len(ls) - len(rs) in (0, 1)
        s = sdim[t]
        v = x[perm[t], s]
        assert all(x[perm[u], s] <= v for u in ls)
        assert all(x[perm[u], s] >= v for u in rs)
        if t > 0:
            assert oracle.parent(t) < t
        if l < n:
            assert oracle.parent(l) == t
        if r < n:
            assert oracle.parent(r) == t


def test_every_prefix_is_parent_closed():
    n = 300
    for t in range(1, n):
        p = oracle.parent(t)
        assert p < t and t in (oracle.left_child(p), oracle.right_child(p))


def test_ties_broken_by_input_index():
    # integer grid: many equal coordinates
    g = np.stack(np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij"), -1).reshape(-1, 3)
    x = g.astype(np.float64)
    perm, sdim = oracle.tree_order(x)
    # root: widest extent ties across all dims -> dim 0; sorted by (x0, index): median rank 13
    order = sorted(range(len(x)), key=lambda i: (x[i, 0], i))
    assert sdim[0] == 0 and perm[0] == order[13]
