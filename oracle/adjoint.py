"""Reverse-mode derivatives of forward, inverse and logdet (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2.3 states that GraphGP provides forward and backward derivatives with
respect to the kernel parameters, built on the Cholesky-derivative formulas of
Smith (1995).  The oracle writes the same derivatives as closed forms of the
conditional formulas of Eq. (2), with F = (I - B)^-1 D as in ``vecchia``:

* forward v = F xi, cotangent v_bar:  w = (I - B)^-T v_bar (reverse sweep),
  xi_bar = D w on the sparse rows, b_bar_i = w_i v[c(i)],
  sigma_bar_i = w_i xi_i; on the dense block g0 = w[0:n0] (cotangent of v0
  including the terms from its children), xi_bar0 = L0^T g0,
  L0_bar = tril(g0 xi0^T).
* inverse xi = F^-1 v, cotangent xi_bar:  z = xi_bar / sigma,
  v_bar = (I - B)^T z on the sparse part plus L0^-T xi_bar0 on the dense block,
  b_bar_i = -z_i v[c(i)], sigma_bar_i = -z_i xi_i, L0_bar = -tril(L0^-T xi_bar0 xi0^T).
* logdet = 2 sum log sigma_i + 2 sum log L0_jj, cotangent ld_bar:
  sigma_bar_i += 2 ld_bar / sigma_i and K0_bar += ld_bar K0^-1.
* per sparse point, with s = sigma_i^2 = K_ii - k^T b, b = K_cc^-1 k,
  sbar = sigma_bar_i / (2 sigma_i) and u = K_cc^-1 b_bar_i:
      theta_bar += sbar dK_ii + sum_p (u_p - 2 sbar b_p) dk_p
                   + sum_{p,q} (sbar b_p b_q - u_p b_q) dK_pq
  (the sum over p, q runs over the full symmetric matrix).
* dense block: with P = Phi(L0^T L0_bar) (lower triangle, diagonal halved),
  S = L0^-T P L0^-1 and K0_bar = (S + S^T)/2 the Cholesky adjoint;
  theta_bar += sum_{p,q} K0_bar_pq dK0_pq.

Coordinates (with_x): at a fixed graph (the order and the neighbour sets are
piecewise constant in x) the same cotangents k_bar_p = u_p - 2 sbar b_p of
k_ci, K_bar_pq = sbar b_p b_q - u_p b_q of K_cc and K0_bar of the dense block
act through d kappa(|x_p - x_q|)/d x_p = kappa'(r) (x_p - x_q)/r on both
points of every entry: x_bar_{c_p} += k_bar_p g(x_{c_p}, x_i),
x_bar_i -= the same, x_bar_{c_p} += sum_q K_bar_pq g(x_{c_p}, x_{c_q}),
x_bar_{c_q} -= the same, and alike for K0.  x_bar is in slot order (N, d).

theta = (sigma, ell).  Pins (tests/test_oracle_adjoint.py): central finite
differences of the oracle's own forward/inverse/logdet, the adjoint
dot-product test <v_bar, F xi> = <F^T v_bar, xi>, d logdet / d sigma = 2N/sigma
without nugget, and in the exact limit d logdet / d ell = tr(K^-1 dK/d ell).
"""
import numpy as np
import scipy.linalg

from .covariance import cov_grad_x, cov_matrix, dkappa_dell, dkappa_dsigma


def _children_scatter(graph, fac, values):
    """acc[j] = sum over (i, m) with c(i)[m] = j of b_i[m] * values[i]."""
    acc = np.zeros(graph.n)
    ok = graph.nbr >= 0
    rows = np.repeat(np.arange(graph.n0, graph.n), graph.k).reshape(graph.nbr.shape)
    np.add.at(acc, graph.nbr[ok], fac.b[ok] * values[rows[ok]])
    return acc


def _cholesky_adjoint(l, l_bar):
    p = np.tril(l.T @ l_bar)
    p[np.diag_indices_from(p)] *= 0.5
    linv = scipy.linalg.solve_triangular(l, np.eye(l.shape[0]), lower=True)
    s = linv.T @ p @ linv
    return 0.5 * (s + s.T)


def theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar):
    """Accumulate (d/dsigma, d/dell) from per-point cotangents of b and sigma
    and the cotangent of the dense-block covariance K0."""
    xs, n0 = graph.xs, graph.n0
    out = np.zeros(2)
    derivs = (("sigma", dkappa_dsigma), ("ell", dkappa_dell))
    for r in range(graph.n - n0):
        row = graph.nbr[r]
        ok = row >= 0
        c = row[ok]
        if len(c) == 0:
            continue
        xc, xi = xs[c], xs[n0 + r][None, :]
        b = fac.b[r][ok]
        sig = fac.sigma[r]
        kcc = cov_matrix(xc, xc, kern, same=True)
        u = np.linalg.solve(kcc, b_bar[r][ok])
        sbar = sigma_bar[r] / (2.0 * sig)
        for t, (name, dk) in enumerate(derivs):
            dkii = float(dk(0.0, kern))
            dkc = cov_matrix(xc, xi, kern, deriv=name)[:, 0]
            dkcc = cov_matrix(xc, xc, kern, deriv=name)
            out[t] += (sbar * dkii + np.sum((u - 2.0 * sbar * b) * dkc)
                       + np.sum((sbar * np.outer(b, b) - np.outer(u, b)) * dkcc))
    x0 = xs[:n0]
    for t, name in enumerate(("sigma", "ell")):
        out[t] += np.sum(k0_bar * cov_matrix(x0, x0, kern, deriv=name))
    return out


def x_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar):
    """Cotangent of the coordinates (slot order, N x d) from the same per-point
    cotangents of b and sigma and the cotangent of K0 as theta_grad."""
    xs, n0 = graph.xs, graph.n0
    out = np.zeros_like(xs, dtype=np.float64)
    for r in range(graph.n - n0):
        row = graph.nbr[r]
        ok = row >= 0
        c = row[ok]
        if len(c) == 0:
            continue
        xc, xi = xs[c], xs[n0 + r][None, :]
        b = fac.b[r][ok]
        kcc = cov_matrix(xc, xc, kern, same=True)
        u = np.linalg.solve(kcc, b_bar[r][ok])
        sbar = sigma_bar[r] / (2.0 * fac.sigma[r])
        k_bar = u - 2.0 * sbar * b
        kcc_bar = sbar * np.outer(b, b) - np.outer(u, b)
        gk = cov_grad_x(xc, xi, kern)[:, 0, :]           # d k_p / d x_{c_p}
        np.add.at(out, c, k_bar[:, None] * gk)
        out[n0 + r] -= np.sum(k_bar[:, None] * gk, axis=0)
        gkk = cov_grad_x(xc, xc, kern)                   # d K_pq / d x_{c_p}
        np.add.at(out, c, np.sum(kcc_bar[:, :, None] * gkk, axis=1))
        np.add.at(out, c, -np.sum(kcc_bar[:, :, None] * gkk, axis=0))
    x0 = xs[:n0]
    g0 = cov_grad_x(x0, x0, kern)
    out[:n0] += np.sum(k0_bar[:, :, None] * g0, axis=1) - np.sum(k0_bar[:, :, None] * g0, axis=0)
    return out


def forward_vjp(graph, fac, kern, xi, v, v_bar, ld_bar=0.0, with_x=False):
    """Cotangents of xi and of (sigma, ell) for the scalar
    <v_bar, v> + ld_bar * logdet, with v = F xi.  Returns (xi_bar, theta_bar),
    and the coordinates' cotangent (slot order) third with with_x."""
    n, n0 = graph.n, graph.n0
    xi = np.asarray(xi, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    v_bar = np.asarray(v_bar, dtype=np.float64)
    w = np.zeros(n)
    acc = np.zeros(n)
    for i in range(n - 1, n0 - 1, -1):                   # reverse generation order
        w[i] = v_bar[i] + acc[i]
        row = graph.nbr[i - n0]
        ok = row >= 0
        np.add.at(acc, row[ok], fac.b[i - n0][ok] * w[i])
    g0 = v_bar[:n0] + acc[:n0]
    xi_bar = np.zeros(n)
    xi_bar[n0:] = fac.sigma * w[n0:]
    xi_bar[:n0] = fac.L0.T @ g0
    gathered = np.where(graph.nbr >= 0, v[np.maximum(graph.nbr, 0)], 0.0)
    b_bar = w[n0:, None] * gathered
    sigma_bar = w[n0:] * xi[n0:] + 2.0 * ld_bar / fac.sigma
    l0_bar = np.tril(np.outer(g0, xi[:n0]))
    k0_bar = _cholesky_adjoint(fac.L0, l0_bar)
    if ld_bar != 0.0:
        k0_bar = k0_bar + ld_bar * scipy.linalg.cho_solve((fac.L0, True), np.eye(n0))
    if with_x:
        return (xi_bar, theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar),
                x_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar))
    return xi_bar, theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar)


def inverse_vjp(graph, fac, kern, v, xi, xi_bar, with_x=False):
    """Cotangents of v and of (sigma, ell) for <xi_bar, xi>, xi = F^-1 v.
    Returns (v_bar, theta_bar), and the coordinates' cotangent third with
    with_x."""
    n0 = graph.n0
    v = np.asarray(v, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    xi_bar = np.asarray(xi_bar, dtype=np.float64)
    z = np.zeros(graph.n)
    z[n0:] = xi_bar[n0:] / fac.sigma
    v_bar = z - _children_scatter(graph, fac, z)
    t0 = scipy.linalg.solve_triangular(fac.L0.T, xi_bar[:n0], lower=False)   # L0^-T xi_bar0
    v_bar[:n0] += t0
    gathered = np.where(graph.nbr >= 0, v[np.maximum(graph.nbr, 0)], 0.0)
    b_bar = -z[n0:, None] * gathered
    sigma_bar = -z[n0:] * xi[n0:]
    l0_bar = -np.tril(np.outer(t0, xi[:n0]))
    k0_bar = _cholesky_adjoint(fac.L0, l0_bar)
    if with_x:
        return (v_bar, theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar),
                x_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar))
    return v_bar, theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar)


def logdet_vjp(graph, fac, kern, ld_bar=1.0, with_x=False):
    """d (ld_bar * logdet) / d (sigma, ell), and with with_x also
    d (ld_bar * logdet) / d x (slot order) second."""
    n0 = graph.n0
    b_bar = np.zeros_like(fac.b)
    sigma_bar = 2.0 * ld_bar / fac.sigma
    k0_bar = ld_bar * scipy.linalg.cho_solve((fac.L0, True), np.eye(n0))
    if with_x:
        return (theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar),
                x_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar))
    return theta_grad(graph, fac, kern, b_bar, sigma_bar, k0_bar)
