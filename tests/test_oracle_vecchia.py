"""Pins of the oracle's factor / forward / inverse / logdet (Eq. (1)-(2), Alg. 1)."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import Kernel, EXP, M32, SE

KERNELS = [Kernel(EXP, 1.0, 0.1), Kernel(M32, 1.3, 0.2), Kernel(SE, 0.8, 0.15, 1e-4)]


def exact_graph(n, seed):
    x = np.random.default_rng(seed).random((n, 3))
    return oracle.build_graph(x, n - 1, 1)      # c(i) = every preceding slot


@pytest.mark.parametrize("kern", KERNELS)
def test_exact_limit_matches_dense_cholesky(kern):
    """Sec. 2.1: conditioning on all preceding points is the dense Cholesky."""
    n = 256
    gr = exact_graph(n, 1)
    fac = oracle.factor(gr, kern)
    kd = oracle.dense_covariance(gr.xs, kern)
    l = np.linalg.cholesky(kd)
    np.testing.assert_allclose(fac.sigma, np.diag(l)[1:], rtol=1e-9)
    # B = I - D L^-1 (rows in slot order)
    bmat = np.eye(n) - np.diag(np.diag(l)) @ scipy.linalg.solve_triangular(l, np.eye(n), lower=True)
    for i in range(1, n):
        row = gr.nbr[i - 1]
        np.testing.assert_allclose(fac.b[i - 1], bmat[i, row], rtol=1e-6, atol=1e-9)
    xi = np.random.default_rng(5).standard_normal(n)
    np.testing.assert_allclose(oracle.forward(gr, fac, xi), l @ xi, rtol=1e-9, atol=1e-9)
    sign, ld = np.linalg.slogdet(kd)
    assert sign > 0
    assert abs(oracle.logdet(fac) - ld) <= 1e-9 * abs(ld)


@pytest.mark.parametrize("n0", [17, 64])
@pytest.mark.parametrize("kern", KERNELS)
def test_exact_limit_with_dense_initial_block(kern, n0):
    """Sec. 2.1 and Sec. 2.2 (dense initial batch): with c(i) = every
    preceding slot, the dense block L0 followed by the sparse rows is the
    dense Cholesky factor of the whole tree-ordered K (nugget on its
    diagonal): L0 is its leading n0 x n0 block, sigma_i its diagonal, the
    forward pass L xi and the logdet slogdet(K).  numpy's Cholesky of the
    full matrix is the independent reference for the dense block."""
    n = 256
    x = np.random.default_rng(7).random((n, 3))
    gr = oracle.build_graph(x, n - 1, n0)
    fac = oracle.factor(gr, kern)
    r = np.sqrt(np.sum((gr.xs[:, None, :] - gr.xs[None, :, :]) ** 2, axis=-1))
    kd = oracle.kappa(r, kern) + kern.nugget * np.eye(n)          # the covariance written out directly
    l = np.linalg.cholesky(kd)
    np.testing.assert_allclose(fac.L0, l[:n0, :n0], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(fac.sigma, np.diag(l)[n0:], rtol=1e-9)
    xi = np.random.default_rng(8).standard_normal(n)
    np.testing.assert_allclose(oracle.forward(gr, fac, xi), l @ xi, rtol=1e-9, atol=1e-9)
    sign, ld = np.linalg.slogdet(kd)
    assert sign > 0
    assert abs(oracle.logdet(fac) - ld) <= 1e-9 * abs(ld)
    np.testing.assert_allclose(oracle.inverse(gr, fac, l @ xi), xi, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("kern", KERNELS)
def test_k1_closed_form(kern):
    x = np.random.default_rng(3).random((50, 3))
    gr = oracle.build_graph(x, 1, 1)
    fac = oracle.factor(gr, kern)
    k00 = kern.sigma ** 2 + kern.nugget
    for i in range(1, 50):
        j = gr.nbr[i - 1, 0]
        r = math.dist(gr.xs[i], gr.xs[j])
        kr = float(oracle.kappa(r, kern))
        assert fac.b[i - 1, 0] == pytest.approx(kr / k00, rel=1e-13)
        assert fac.sigma[i - 1] == pytest.approx(math.sqrt(k00 - kr * kr / k00), rel=1e-12)


def test_homogeneity_in_sigma():
    x = np.random.default_rng(4).random((300, 3))
    gr = oracle.build_graph(x, 8, 16)
    f1 = oracle.factor(gr, Kernel(M32, 1.0, 0.1))
    f3 = oracle.factor(gr, Kernel(M32, 3.0, 0.1))
    np.testing.assert_allclose(f3.b, f1.b, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(f3.sigma, 3.0 * f1.sigma, rtol=1e-12)
    assert oracle.logdet(f3) == pytest.approx(oracle.logdet(f1) + 2 * 300 * math.log(3.0), rel=1e-12)


def test_permuting_conditioning_set():
    rng = np.random.default_rng(6)
    xc, xi = rng.random((12, 3)), rng.random(3)
    kern = Kernel(EXP, 1.0, 0.3)
    b, s = oracle.conditional(xc, xi, kern)
    p = rng.permutation(12)
    bp, sp = oracle.conditional(xc[p], xi, kern)
    np.testing.assert_allclose(bp, b[p], rtol=1e-10)
    assert sp == pytest.approx(s, rel=1e-13)


@pytest.mark.parametrize("kern", KERNELS)
def test_joint_form_of_alg1_agrees_with_eq2(kern):
    rng = np.random.default_rng(8)
    for _ in range(20):
        xc, xi = rng.random((16, 3)), rng.random(3)
        b1, s1 = oracle.conditional(xc, xi, kern)
        b2, s2 = oracle.conditional_joint(xc, xi, kern)
        assert abs(s1 - s2) <= 1e-13 * max(1.0, s1) * 10
        np.testing.assert_allclose(b1, b2, rtol=1e-9, atol=1e-12)


def test_batched_factor_equals_per_point():
    x = np.random.default_rng(9).random((400, 3))
    gr = oracle.build_graph(x, 8, 4)          # n0 < k: first rows padded
    kern = Kernel(M32, 1.0, 0.1)
    fac = oracle.factor(gr, kern)
    for r in (0, 1, 3, 4, 100, 395):
        row = gr.nbr[r]
        ok = row >= 0
        b, s = oracle.conditional(gr.xs[row[ok]], gr.xs[4 + r], kern)
        np.testing.assert_allclose(fac.b[r][ok], b, rtol=1e-9, atol=1e-13)
        assert (fac.b[r][~ok] == 0).all()
        assert fac.sigma[r] == pytest.approx(s, rel=1e-12)


@pytest.mark.parametrize("kern", KERNELS)
def test_forward_routes_agree(kern):
    x = np.random.default_rng(10).random((700, 3))
    gr = oracle.build_graph(x, 8, 32)
    fac = oracle.factor(gr, kern)
    xi = np.random.default_rng(11).standard_normal(700)
    v = oracle.forward(gr, fac, xi)
    np.testing.assert_allclose(v, oracle.forward_sequential(gr, fac, xi), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(v, oracle.forward_sparse_solve(gr, fac, xi), rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("kern", KERNELS)
def test_inverse_round_trip(kern):
    x = np.random.default_rng(12).random((500, 3))
    gr = oracle.build_graph(x, 16, 20)
    fac = oracle.factor(gr, kern)
    xi = np.random.default_rng(13).standard_normal(500)
    np.testing.assert_allclose(oracle.inverse(gr, fac, oracle.forward(gr, fac, xi)), xi, atol=1e-8)


@pytest.mark.parametrize("kern", KERNELS)
def test_logdet_equals_sparse_precision_slogdet(kern):
    n = 200
    x = np.random.default_rng(14).random((n, 3))
    gr = oracle.build_graph(x, 6, 10)
    fac = oracle.factor(gr, kern)
    m, d = oracle.vecchia.sparse_factor_matrices(gr, fac)
    q = m.toarray().T @ np.diag(d ** -2) @ m.toarray()
    sign, ld = np.linalg.slogdet(q)
    assert sign > 0
    assert oracle.logdet(fac) == pytest.approx(-ld, rel=1e-9)


def test_not_positive_definite_reports_slot():
    x = np.random.default_rng(15).random((40, 3))
    x[30] = x[3]                       # duplicate point, no nugget
    gr = oracle.build_graph(x, 8, 8)
    with pytest.raises(oracle.vecchia.NotPositiveDefinite) as e:
        oracle.factor(gr, Kernel(SE, 1.0, 0.2))
    assert e.value.slot >= 8
