"""Forward-mode derivatives (tangents) of forward and logdet (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2.3 states that GraphGP provides forward as well as backward
derivatives with respect to the kernel parameters.  For a direction
(xi_dot, theta_dot), theta = (sigma, ell), and K_dot = sum_t theta_dot_t
dK/dtheta_t (nugget excluded), differentiating Eq. (2) gives, per sparse
point with b = K_cc^-1 k_ci and sigma^2 = K_ii - k_ci . b:

    b_dot       = K_cc^-1 (k_dot_ci - K_dot_cc b)
    (sigma^2)'  = K_dot_ii - 2 k_dot_ci . b + b . K_dot_cc b
    sigma_dot   = (sigma^2)' / (2 sigma)

and differentiating Alg. 1's recursion v_i = b . v[c(i)] + sigma_i xi_i:

    v_dot_i = b_dot . v[c(i)] + b . v_dot[c(i)] + sigma_dot_i xi_i + sigma_i xi_dot_i,

batch by batch.  The dense block v0 = L0 xi0 has v0_dot = L0_dot xi0 +
L0 xi0_dot with the Cholesky tangent L0_dot = L0 Phi(L0^-1 K0_dot L0^-T)
(Phi: lower triangle with the diagonal halved).  The logdet tangent is
2 sum sigma_dot_i / sigma_i + tr(K0^-1 K0_dot).

Pins (tests/test_oracle_tangent.py): central finite differences of the
oracle's own forward and logdet, and the pairing with the reverse mode,
<v_bar, J theta_dot> = <J^T v_bar, theta_dot> and <v_bar, F xi_dot> =
<F^T v_bar, xi_dot>, using ``oracle.adjoint``.
"""
import numpy as np
import scipy.linalg

from .covariance import cov_matrix, dkappa_dell, dkappa_dsigma


def _k_dot(xa, xb, kern, theta_dot):
    """Directional derivative of kappa(|xa - xb|) (no nugget)."""
    return (theta_dot[0] * cov_matrix(xa, xb, kern, deriv="sigma")
            + theta_dot[1] * cov_matrix(xa, xb, kern, deriv="ell"))


def factor_tangent(graph, fac, kern, theta_dot):
    """(b_dot (Ns, k), sigma_dot (Ns,), L0_dot (n0, n0)) for the direction theta_dot."""
    xs, n0 = graph.xs, graph.n0
    theta_dot = np.asarray(theta_dot, dtype=np.float64)
    b_dot = np.zeros_like(fac.b)
    sigma_dot = np.zeros_like(fac.sigma)
    kii_dot = theta_dot[0] * float(dkappa_dsigma(0.0, kern)) + theta_dot[1] * float(dkappa_dell(0.0, kern))
    for r in range(graph.n - n0):
        row = graph.nbr[r]
        ok = row >= 0
        c = row[ok]
        b = fac.b[r][ok]
        xc, xi = xs[c], xs[n0 + r][None, :]
        kcc = cov_matrix(xc, xc, kern, same=True)
        kdc = _k_dot(xc, xi, kern, theta_dot)[:, 0]
        kdcc = _k_dot(xc, xc, kern, theta_dot)
        b_dot[r][ok] = np.linalg.solve(kcc, kdc - kdcc @ b) if len(c) else 0.0
        s2_dot = kii_dot - 2.0 * kdc @ b + b @ kdcc @ b
        sigma_dot[r] = s2_dot / (2.0 * fac.sigma[r])
    l0 = fac.L0
    x0 = xs[:n0]
    k0_dot = _k_dot(x0, x0, kern, theta_dot)
    linv = scipy.linalg.solve_triangular(l0, np.eye(n0), lower=True)
    x = linv @ k0_dot @ linv.T
    phi = np.tril(x)
    phi[np.diag_indices_from(phi)] *= 0.5
    return b_dot, sigma_dot, l0 @ phi, float(np.trace(x))


def forward_jvp(graph, fac, kern, xi, xi_dot, theta_dot):
    """(v_dot, logdet_dot) of v = F(xi; theta) in the direction (xi_dot, theta_dot)."""
    n0 = graph.n0
    xi = np.asarray(xi, dtype=np.float64)
    xi_dot = np.asarray(xi_dot, dtype=np.float64)
    b_dot, sigma_dot, l0_dot, tr0 = factor_tangent(graph, fac, kern, theta_dot)
    v = np.zeros(graph.n)
    vd = np.zeros(graph.n)
    v[:n0] = fac.L0 @ xi[:n0]
    vd[:n0] = l0_dot @ xi[:n0] + fac.L0 @ xi_dot[:n0]
    for level in range(1, graph.n_levels + 1):
        rows = graph.level_slots(level) - n0
        nb = graph.nbr[rows]
        ok = nb >= 0
        gv = np.where(ok, v[np.maximum(nb, 0)], 0.0)
        gd = np.where(ok, vd[np.maximum(nb, 0)], 0.0)
        s = n0 + rows
        v[s] = np.sum(fac.b[rows] * gv, axis=1) + fac.sigma[rows] * xi[s]
        vd[s] = (np.sum(b_dot[rows] * gv, axis=1) + np.sum(fac.b[rows] * gd, axis=1)
                 + sigma_dot[rows] * xi[s] + fac.sigma[rows] * xi_dot[s])
    ld_dot = 2.0 * float(np.sum(sigma_dot / fac.sigma)) + tr0
    return vd, ld_dot
