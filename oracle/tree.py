"""Bit-reversed, left-balanced k-d tree order (Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2.2, "Bit-reversed ordering": the node in slot t at tree level
l = floor(log2(t+1)) has its left child in slot t + 2^l and its right child in
slot t + 2^(l+1) (0-based slots).  A child exists iff its slot is < N.  With
every level full this is a bit-reversal permutation of each level of the usual
heap order; with a partial last level, the last level is filled in
bit-reversed position order.  Consequences used below (derived, not printed):

* every level except the last is full;
* at every node |left subtree| - |right subtree| is 0 or 1, so the node that
  owns a subset S of size n keeps the element of sorted rank m = floor(n/2)
  (= ceil((n-1)/2)), the left child gets the m smaller elements and the right
  child the rest ("left-balanced", Sec. 2.2 "Tree ordering");
* parent(t) < t, so every prefix {0..i-1} is itself such a tree.

Readings where the paper is silent:

* split dimension: the dimension of widest extent (max - min) of the node's
  subset, lowest dimension on ties;
* order inside a node: sort by (coordinate on the split dimension, input
  index), so equal coordinates are ordered by input index.

Pins (tests/test_oracle_tree.py): for N = 2^L - 1 the order equals the usual
heap-order median tree with each level bit-reversed; a hand-derived fixture
(tests/golden/tree_1d_n10.json); the k-d property, the balance property and
parent closure at ragged N.
"""
import numpy as np


def tree_level(t):
    return (int(t) + 1).bit_length() - 1


def left_child(t):
    return t + (1 << tree_level(t))


def right_child(t):
    return t + (1 << (tree_level(t) + 1))


def parent(t):
    """Slot of the parent of slot t >= 1 (inverse of the child formula)."""
    l = tree_level(t)
    q = t - ((1 << l) - 1)          # position inside level l
    half = 1 << (l - 1)
    q_parent = q % half
    return (half - 1) + q_parent


def split_dim(points):
    ext = points.max(axis=0) - points.min(axis=0)
    return int(np.argmax(ext))      # first maximum -> lowest dimension on ties


def tree_order(x):
    """Return (perm, sdim): perm[t] = input index placed in slot t, sdim[t] =
    split dimension used at slot t (0 for leaves, whose extent is all zero)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n = x.shape[0]
    perm = np.full(n, -1, dtype=np.int64)
    sdim = np.zeros(n, dtype=np.int64)
    stack = [(0, np.arange(n, dtype=np.int64))]
    while stack:
        t, subset = stack.pop()
        s = split_dim(x[subset])
        order = np.lexsort((subset, x[subset, s]))   # key: (coordinate, input index)
        subset = subset[order]
        m = len(subset) // 2
        perm[t] = subset[m]
        sdim[t] = s
        left, right = left_child(t), right_child(t)
        if m > 0:
            assert left < n
            stack.append((left, subset[:m]))
        else:
            assert left >= n
        if len(subset) - m - 1 > 0:
            assert right < n
            stack.append((right, subset[m + 1:]))
        else:
            assert right >= n
    assert (perm >= 0).all()
    return perm, sdim
