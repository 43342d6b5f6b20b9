"""The order/accuracy study's host parts (paper_2606_11402_amd/study.py):
batch sizes from the graph, and its KL formula
    KL = 1/2 [ || D^-1 (I - B) L_K ||_F^2 - N + log det K~ - log det K ]
checked against the textbook dense formula
    KL = 1/2 [ tr(K~^-1 K) - N + log det K~ - log det K ],  K~ = F F^T,
with the oracle's factor (FP64) on small clouds."""
import numpy as np
import pytest

import oracle
from oracle import Kernel, M32, M52, SE
from paper_2606_11402_amd import Graph, KernelParams
from paper_2606_11402_amd import study


def test_batch_sizes_partition_the_sparse_points():
    x = np.random.default_rng(1).standard_normal((3000, 3))
    g = Graph(x, 16, 50)
    bs = study.batch_sizes(g)
    assert len(bs) == g.n_levels and (bs > 0).all() and bs.sum() == g.n - g.n0


def device_rows_from_oracle(g, og, of):
    """The oracle's coefficients laid out like the device rows: for every
    storage position's sparse row, the neighbours in ascending storage
    position (the graph's tiled layout), b permuted alike."""
    n0, kp = g.n0, g.kp
    ns = g.n - n0
    pos = np.empty(g.n, dtype=np.int64)
    pos[g.slot] = np.arange(g.n)                     # slot -> storage position
    b_dev = np.zeros((ns, kp))
    nbr = g.nbr(1).reshape(g.ntiles, kp, 64).transpose(0, 2, 1).reshape(-1, kp)[:ns]
    for sp in range(ns):
        slot = g.slot[n0 + sp]
        row = og.nbr[slot - n0]
        ok = row >= 0
        p = pos[row[ok]]
        order = np.argsort(p)
        assert (nbr[sp][:ok.sum()] == p[order]).all()
        b_dev[sp, :ok.sum()] = of.b[slot - n0][ok][order]
    sigma = np.array([of.sigma[g.slot[n0 + sp] - n0] for sp in range(ns)])
    return b_dev, sigma


@pytest.mark.parametrize("kind,k,n0", [(M32, 4, 20), (SE, 8, 1), (M52, 16, 32)])
def test_kl_formula_matches_the_dense_definition(kind, k, n0):
    n = 300
    x = np.random.default_rng(kind + k).standard_normal((n, 3))
    kern = Kernel(kind, 1.0, 1.0, 1e-6)
    g = Graph(x, k, n0)
    og = oracle.build_graph(x, k, n0)
    of = oracle.factor(og, kern)
    b_dev, sigma = device_rows_from_oracle(g, og, of)
    lk, ld_k = study.exact_cholesky(x, KernelParams(kind, 1.0, 1.0, 1e-6))
    pos = np.empty(g.n, dtype=np.int64)
    pos[g.order] = np.arange(g.n)
    m = study.precision_factor(g, b_dev, sigma, of.L0)[:, pos]
    y = m @ lk
    kl_study = 0.5 * (np.sum(y * y) - n + oracle.logdet(of) - ld_k)
    # textbook: dense K~ = F F^T in slot order, K in slot order
    mat, d = oracle.vecchia.sparse_factor_matrices(og, of)
    f = np.linalg.solve(mat.toarray(), np.diag(d))
    kt = f @ f.T
    kd = oracle.dense_covariance(og.xs, kern)
    kl_ref = 0.5 * (np.trace(np.linalg.solve(kt, kd)) - n + np.linalg.slogdet(kt)[1] - np.linalg.slogdet(kd)[1])
    assert kl_ref > 0
    assert abs(kl_study - kl_ref) <= 1e-7 * max(1.0, abs(kl_ref)), (kl_study, kl_ref)
