"""Pins of the oracle's derivatives: finite differences, dot-product tests and
closed forms."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import Kernel, EXP, M32, SE


def loss_fwd(gr, kern, xi, y, s2):
    fac = oracle.factor(gr, kern)
    v = oracle.forward(gr, fac, xi)
    return 0.5 * np.sum((v - y) ** 2) / s2 + oracle.logdet(fac)


def small_case(seed, n=120, k=6, n0=12):
    rng = np.random.default_rng(seed)
    gr = oracle.build_graph(rng.random((n, 3)), k, n0)
    return gr, rng.standard_normal(n), rng.standard_normal(n)


@pytest.mark.parametrize("kind", [EXP, M32, SE])
def test_forward_loss_theta_gradient_central_difference(kind):
    gr, xi, y = small_case(1)
    kern = Kernel(kind, 1.2, 0.25, 1e-3 if kind == SE else 0.0)
    s2 = 0.1 ** 2
    fac = oracle.factor(gr, kern)
    v = oracle.forward(gr, fac, xi)
    _, g = oracle.forward_vjp(gr, fac, kern, xi, v, (v - y) / s2, ld_bar=1.0)
    h = 1e-5                     # central difference truncation ~ h^2: 1e-8 relative here
    for t, name in enumerate(("sigma", "ell")):
        kp = Kernel(kind, kern.sigma + h * (t == 0), kern.ell + h * (t == 1), kern.nugget)
        km = Kernel(kind, kern.sigma - h * (t == 0), kern.ell - h * (t == 1), kern.nugget)
        fd = (loss_fwd(gr, kp, xi, y, s2) - loss_fwd(gr, km, xi, y, s2)) / (2 * h)
        assert g[t] == pytest.approx(fd, rel=1e-6, abs=1e-6), name


def test_forward_xi_gradient_central_difference():
    gr, xi, y = small_case(2)
    kern = Kernel(M32, 1.0, 0.2)
    fac = oracle.factor(gr, kern)
    v = oracle.forward(gr, fac, xi)
    s2 = 0.01
    gxi, _ = oracle.forward_vjp(gr, fac, kern, xi, v, (v - y) / s2, ld_bar=1.0)
    h = 1e-4
    for j in (0, 5, 11, 12, 60, 119):
        e = np.zeros_like(xi)
        e[j] = h
        fd = (loss_fwd(gr, kern, xi + e, y, s2) - loss_fwd(gr, kern, xi - e, y, s2)) / (2 * h)
        assert gxi[j] == pytest.approx(fd, rel=1e-7, abs=1e-6)


def test_forward_adjoint_dot_product():
    gr, xi, vbar = small_case(3)
    kern = Kernel(EXP, 1.0, 0.1)
    fac = oracle.factor(gr, kern)
    v = oracle.forward(gr, fac, xi)
    ft_vbar, _ = oracle.forward_vjp(gr, fac, kern, xi, v, vbar)
    assert np.dot(vbar, v) == pytest.approx(np.dot(ft_vbar, xi), rel=1e-12)


def test_inverse_vjp_dot_product_and_fd():
    gr, v, xibar = small_case(4)
    kern = Kernel(M32, 0.9, 0.3)
    fac = oracle.factor(gr, kern)
    xi = oracle.inverse(gr, fac, v)
    vbar, g = oracle.inverse_vjp(gr, fac, kern, v, xi, xibar)
    assert np.dot(xibar, xi) == pytest.approx(np.dot(vbar, v), rel=1e-11)
    h = 1e-5

    def f(kp):
        return np.dot(xibar, oracle.inverse(gr, oracle.factor(gr, kp), v))

    for t in range(2):
        kp = Kernel(M32, kern.sigma + h * (t == 0), kern.ell + h * (t == 1))
        km = Kernel(M32, kern.sigma - h * (t == 0), kern.ell - h * (t == 1))
        assert g[t] == pytest.approx((f(kp) - f(km)) / (2 * h), rel=1e-6, abs=1e-6)


def test_dlogdet_dsigma_is_2n_over_sigma():
    gr, _, _ = small_case(5)
    kern = Kernel(SE, 1.7, 0.2)
    fac = oracle.factor(gr, kern)
    g = oracle.logdet_vjp(gr, fac, kern, 1.0)
    assert g[0] == pytest.approx(2 * gr.n / 1.7, rel=1e-10)


@pytest.mark.parametrize("kind", [EXP, M32])
def test_exact_limit_dlogdet_dell_is_trace(kind):
    n = 60
    x = np.random.default_rng(6).random((n, 3))
    gr = oracle.build_graph(x, n - 1, 1)
    kern = Kernel(kind, 1.0, 0.2)
    fac = oracle.factor(gr, kern)
    g = oracle.logdet_vjp(gr, fac, kern, 1.0)
    kd = oracle.dense_covariance(gr.xs, kern)
    dk = oracle.cov_matrix(gr.xs, gr.xs, kern, deriv="ell")
    assert g[1] == pytest.approx(np.trace(np.linalg.solve(kd, dk)), rel=1e-8)


def test_dense_block_only_gradient():
    """n0 = N: the whole field is the dense block; the Cholesky adjoint alone
    must match finite differences."""
    gr, xi, y = small_case(7, n=40, k=4, n0=40)
    kern = Kernel(M32, 1.1, 0.3)
    fac = oracle.factor(gr, kern)
    v = oracle.forward(gr, fac, xi)
    _, g = oracle.forward_vjp(gr, fac, kern, xi, v, (v - y), ld_bar=1.0)
    h = 1e-5
    for t in range(2):
        kp = Kernel(M32, kern.sigma + h * (t == 0), kern.ell + h * (t == 1))
        km = Kernel(M32, kern.sigma - h * (t == 0), kern.ell - h * (t == 1))
        fd = (loss_fwd(gr, kp, xi, y, 1.0) - loss_fwd(gr, km, xi, y, 1.0)) / (2 * h)
        assert g[t] == pytest.approx(fd, rel=1e-6)
