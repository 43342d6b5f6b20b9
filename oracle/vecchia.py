"""Vecchia factor, forward generation, inverse application and log-determinant.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Everything is FP64 and
indexed by tree slot (``oracle.graph.Graph``).

* Eq. (1)-(2): v_i | v_c ~ N(K_ic K_cc^-1 v_c, K_ii - K_ic K_cc^-1 K_ci).  With
  K_cc = L L^T, y = L^-1 k_ci, the coefficients are b_i = L^-T y and the
  conditional standard deviation is sigma_i = sqrt(K_ii - y.y)
  (``conditional``).  Alg. 1 writes the same thing as the Cholesky factor of
  the joint (k+1)x(k+1) covariance with point i last: its last row is
  (y^T, sigma_i) (``conditional_joint``).
* Dense initial batch (Sec. 2.2, Alg. 1): v[0:n0] = chol(K[0:n0,0:n0]) xi[0:n0].
* Forward (Alg. 1): batch by batch, v_i = b_i . v[c(i)] + sigma_i xi_i.
  Writing B for the strictly lower matrix with row i = b_i at the columns c(i)
  and D = diag(sigma), this is v = F xi with F = (I - B)^-1 D; for the dense
  block (I - B0)^-1 D0 = L0.  Sec. 2.1 notes the precision is sparse: the
  forward pass is a sparse triangular solve (``forward_sparse_solve``).
* Inverse application (abstract): xi = F^-1 v, i.e.
  xi[0:n0] = L0^-1 v[0:n0] and xi_i = (v_i - b_i . v[c(i)]) / sigma_i.
* Log-determinant (abstract): log det(F F^T) = 2 (sum_j log L0_jj +
  sum_i log sigma_i), summed with math.fsum.

Pins (tests/test_oracle_vecchia.py): with c(i) = all preceding points the
factor equals the dense Cholesky of K (Sec. 2.1, exact limit): sigma_i = L_ii,
F = L, logdet = numpy slogdet; k = 1 closed form; homogeneity in sigma;
invariance under permutation of c(i); the joint and the conditional forms
agree; forward equals the scipy sparse triangular solve; the inverse undoes
the forward; logdet equals -slogdet of the sparse precision.
"""
import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from .covariance import cov_matrix, kappa


class NotPositiveDefinite(ArithmeticError):
    def __init__(self, slot):
        super().__init__("covariance not positive definite at slot %d" % slot)
        self.slot = slot


@dataclass
class Factor:
    L0: np.ndarray       # (n0, n0) lower Cholesky factor of the dense block
    b: np.ndarray        # (N - n0, k) coefficients, 0 at padded entries
    sigma: np.ndarray    # (N - n0,) conditional standard deviations


def dense_covariance(xs, kern):
    return cov_matrix(xs, xs, kern, same=True)


def dense_block(xs, n0, kern):
    k0 = dense_covariance(np.asarray(xs)[:n0], kern)
    try:
        return np.linalg.cholesky(k0)
    except np.linalg.LinAlgError:
        raise NotPositiveDefinite(0)


def conditional(xc, xi, kern, slot=-1):
    """Eq. (2) through the Cholesky factor of K_cc: returns (b, sigma)."""
    xc = np.atleast_2d(np.asarray(xc, dtype=np.float64))
    xi = np.asarray(xi, dtype=np.float64).reshape(1, -1)
    kcc = cov_matrix(xc, xc, kern, same=True)
    kci = cov_matrix(xc, xi, kern)[:, 0]
    kii = float(kappa(0.0, kern)) + kern.nugget
    try:
        lc = np.linalg.cholesky(kcc)
    except np.linalg.LinAlgError:
        raise NotPositiveDefinite(slot)
    y = scipy.linalg.solve_triangular(lc, kci, lower=True)
    b = scipy.linalg.solve_triangular(lc.T, y, lower=False)
    s = kii - y @ y
    if not s > 0.0:
        raise NotPositiveDefinite(slot)
    return b, math.sqrt(s)


def conditional_joint(xc, xi, kern):
    """Alg. 1: Cholesky of the joint covariance of [c(i), i]; the last row is
    (y^T, sigma_i) and b = L_cc^-T y.  Returns (b, sigma)."""
    xc = np.atleast_2d(np.asarray(xc, dtype=np.float64))
    xj = np.vstack([xc, np.asarray(xi, dtype=np.float64).reshape(1, -1)])
    lj = np.linalg.cholesky(cov_matrix(xj, xj, kern, same=True))
    y = lj[-1, :-1]
    b = scipy.linalg.solve_triangular(lj[:-1, :-1].T, y, lower=False)
    return b, float(lj[-1, -1])


def _batched_conditional(xc, xi, kern, slots):
    """Eq. (2) for a stack of points with full rows: xc (m, k, d), xi (m, d).
    Cholesky by numpy on the stack; the two triangular solves written out as
    plain forward and backward substitution over the k unknowns."""
    m, k, _ = xc.shape
    diff = xc[:, :, None, :] - xc[:, None, :, :]
    kcc = kappa(np.sqrt(np.sum(diff * diff, axis=-1)), kern) + kern.nugget * np.eye(k)
    dci = xc - xi[:, None, :]
    kci = kappa(np.sqrt(np.sum(dci * dci, axis=-1)), kern)
    kii = float(kappa(0.0, kern)) + kern.nugget
    try:
        lc = np.linalg.cholesky(kcc)
    except np.linalg.LinAlgError:
        for j in range(m):     # find the first failing point
            conditional(xc[j], xi[j], kern, slot=int(slots[j]))
        raise
    y = np.zeros((m, k))
    for j in range(k):
        y[:, j] = (kci[:, j] - np.sum(lc[:, j, :j] * y[:, :j], axis=1)) / lc[:, j, j]
    b = np.zeros((m, k))
    for j in range(k - 1, -1, -1):
        b[:, j] = (y[:, j] - np.sum(lc[:, j + 1:, j] * b[:, j + 1:], axis=1)) / lc[:, j, j]
    s = kii - np.sum(y * y, axis=1)
    bad = np.nonzero(~(s > 0.0))[0]
    if len(bad):
        raise NotPositiveDefinite(int(slots[bad[0]]))
    return b, np.sqrt(s)


def factor(graph, kern, rows=None, chunk=4096):
    """Coefficients and conditional standard deviations of every sparse slot
    (or of the sparse rows listed in ``rows``, indices into 0..N-n0-1), plus
    the dense-block factor L0."""
    n0, k = graph.n0, graph.k
    xs = graph.xs
    l0 = dense_block(xs, n0, kern)
    rows = np.arange(graph.n - n0) if rows is None else np.asarray(rows, dtype=np.int64)
    b = np.zeros((len(rows), k))
    sigma = np.zeros(len(rows))
    nbr = graph.nbr[rows]
    full = np.all(nbr >= 0, axis=1)
    for j in np.nonzero(~full)[0]:                      # points with < k predecessors
        row = nbr[j][nbr[j] >= 0]
        bj, sj = conditional(xs[row], xs[n0 + rows[j]], kern, slot=int(n0 + rows[j]))
        b[j, :len(row)] = bj
        sigma[j] = sj
    idx = np.nonzero(full)[0]
    for a in range(0, len(idx), chunk):
        sel = idx[a:a + chunk]
        bj, sj = _batched_conditional(xs[nbr[sel]], xs[n0 + rows[sel]], kern, n0 + rows[sel])
        b[sel] = bj
        sigma[sel] = sj
    return Factor(L0=l0, b=b, sigma=sigma)


def _level_rows(graph):
    for level in range(1, graph.n_levels + 1):
        yield graph.level_slots(level) - graph.n0


def forward(graph, fac, xi):
    """Alg. 1: dense initial batch, then the parallel batches in depth order."""
    n0 = graph.n0
    xi = np.asarray(xi, dtype=np.float64)
    v = np.zeros(graph.n)
    v[:n0] = fac.L0 @ xi[:n0]
    for rows in _level_rows(graph):
        nb = graph.nbr[rows]
        gathered = np.where(nb >= 0, v[np.maximum(nb, 0)], 0.0)
        v[n0 + rows] = np.sum(fac.b[rows] * gathered, axis=1) + fac.sigma[rows] * xi[n0 + rows]
    return v


def forward_sequential(graph, fac, xi):
    """Eq. (1) read literally: v_i drawn one after the other in slot order."""
    n0 = graph.n0
    v = np.zeros(graph.n)
    v[:n0] = fac.L0 @ np.asarray(xi[:n0], dtype=np.float64)
    for i in range(n0, graph.n):
        row = graph.nbr[i - n0]
        ok = row >= 0
        v[i] = fac.b[i - n0][ok] @ v[row[ok]] + fac.sigma[i - n0] * xi[i]
    return v


def sparse_factor_matrices(graph, fac):
    """(I - B) as a scipy CSR matrix and the diagonal D, dense block folded in
    through (I - B0) = D0 L0^-1."""
    n, n0 = graph.n, graph.n0
    d0 = np.diag(fac.L0).copy()
    i_minus_b0 = d0[:, None] * scipy.linalg.solve_triangular(fac.L0, np.eye(n0), lower=True)
    rows, cols, vals = [], [], []
    r0, c0 = np.nonzero(np.tril(np.ones((n0, n0))))
    rows.append(r0), cols.append(c0), vals.append(i_minus_b0[r0, c0])
    ns = n - n0
    rows.append(np.arange(n0, n)), cols.append(np.arange(n0, n)), vals.append(np.ones(ns))
    ok = graph.nbr >= 0
    rr = np.repeat(np.arange(n0, n), graph.k).reshape(ns, graph.k)
    rows.append(rr[ok]), cols.append(graph.nbr[ok]), vals.append(-fac.b[ok])
    m = scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(n, n))
    return m, np.concatenate([d0, fac.sigma])


def forward_sparse_solve(graph, fac, xi):
    """Sec. 2.1: dense covariance, sparse precision -- solve (I - B) v = D xi."""
    m, d = sparse_factor_matrices(graph, fac)
    return scipy.sparse.linalg.spsolve_triangular(m, d * np.asarray(xi, dtype=np.float64), lower=True)


def inverse(graph, fac, v):
    n0 = graph.n0
    v = np.asarray(v, dtype=np.float64)
    xi = np.zeros(graph.n)
    xi[:n0] = scipy.linalg.solve_triangular(fac.L0, v[:n0], lower=True)
    nb = graph.nbr
    gathered = np.where(nb >= 0, v[np.maximum(nb, 0)], 0.0)
    xi[n0:] = (v[n0:] - np.sum(fac.b * gathered, axis=1)) / fac.sigma
    return xi


def logdet(fac):
    terms = [math.log(x) for x in np.diag(fac.L0)] + [math.log(x) for x in fac.sigma]
    return 2.0 * math.fsum(terms)
