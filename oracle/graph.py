"""Conditioning graph: k nearest preceding neighbours, depths, parallel batches.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Neighbours (Sec. 2.1): c(i) is the set of the k nearest points among the
  points that precede i in the generation order (the slots of the bit-reversed
  tree, ``oracle.tree``).  Brute force over all j < i.
  Readings: the squared distance is computed in FP64 as
  ((dx*dx + dy*dy) + dz*dz) with dx = x_i - x_j and no fused multiply-add
  (fewer terms for d < 3); ties are broken by the smaller slot, so the key is
  (D, j); a row lists its neighbours in ascending key order; a slot i with
  fewer than k predecessors keeps all of them and pads the row with -1.
* Dense initial batch (Sec. 2.2, "Batch construction"): slots 0..n0-1 are
  generated jointly by a dense Cholesky factor; they carry depth 0 and no
  neighbour row.
* Depth (Sec. 2.2, "Batch construction"): d_i = 1 + max_{j in c(i)} d_j,
  evaluated in slot order; points of equal depth form one parallel batch.
* Canonical storage order: stable sort of the slots by (depth, slot), so the
  dense block comes first and every batch is contiguous.  Any order that keeps
  the batches contiguous and in increasing depth leaves every conditioning
  relationship unchanged.

Pins (tests/test_oracle_graph.py): neighbour sets and distances against
scipy.spatial.cKDTree queried on each prefix; a hand-derived fixture with ties
(tests/golden/graph_1d_n10.json); the depth invariants.
"""
from dataclasses import dataclass

import numpy as np

from .tree import tree_order


def squared_distances(xs_prefix, xi):
    """FP64 squared distances, summed left to right over the dimensions."""
    diff = xi[None, :] - xs_prefix
    d2 = diff[:, 0] * diff[:, 0]
    for c in range(1, diff.shape[1]):
        d2 = d2 + diff[:, c] * diff[:, c]
    return d2


def preceding_knn(xs, k, n0):
    """Neighbour rows for slots n0..N-1 of points xs given in slot order.
    Returns int64 array (N - n0, k) of slots, padded with -1."""
    xs = np.asarray(xs, dtype=np.float64)
    n = xs.shape[0]
    nbr = np.full((n - n0, k), -1, dtype=np.int64)
    for i in range(n0, n):
        d2 = squared_distances(xs[:i], xs[i])
        order = np.argsort(d2, kind="stable")[:min(k, i)]   # stable: equal D -> smaller slot
        nbr[i - n0, :len(order)] = order
    return nbr


def depths(nbr, n, n0):
    d = np.zeros(n, dtype=np.int64)
    for i in range(n0, n):
        row = nbr[i - n0]
        row = row[row >= 0]
        d[i] = 1 + d[row].max()
    return d


def storage_order(depth):
    """Storage position -> slot, stable by (depth, slot)."""
    return np.argsort(depth, kind="stable")


@dataclass
class Graph:
    n: int
    k: int
    n0: int
    perm: np.ndarray        # slot -> input index
    sdim: np.ndarray        # slot -> split dimension
    xs: np.ndarray          # coordinates in slot order (N, d)
    nbr: np.ndarray         # (N - n0, k) neighbour slots of slots n0..N-1, -1 padded
    depth: np.ndarray       # slot -> depth (0 for the dense block)
    order: np.ndarray       # storage position -> slot, stable by (depth, slot)

    @property
    def n_levels(self):
        return int(self.depth.max()) if self.n > self.n0 else 0

    def level_slots(self, level):
        return np.nonzero(self.depth == level)[0]


def build_graph(x, k, n0):
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n = x.shape[0]
    if not (1 <= n0 <= n):
        raise ValueError("need 1 <= n0 <= N")
    perm, sdim = tree_order(x)
    xs = x[perm]
    nbr = preceding_knn(xs, k, n0)
    depth = depths(nbr, n, n0)
    return Graph(n=n, k=k, n0=n0, perm=perm, sdim=sdim, xs=xs, nbr=nbr,
                 depth=depth, order=storage_order(depth))
