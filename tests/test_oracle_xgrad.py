"""Pins of the oracle's coordinate derivatives (with_x): the distance
derivative of every kernel against a central difference, the full cotangent
of the coordinates of the forward / inverse / logdet losses against central
differences of the oracle's own losses at a fixed graph (order and
neighbour sets held, as the derivative is defined), and, in the exact limit
k = N - 1, the logdet's coordinate gradient against the dense closed form
d log det K / d x_p = 2 sum_q (K^-1)_pq d K_pq / d x_p."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import Kernel, EXP, M32, SE, M52


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
def test_dkappa_dr_central_difference(kind):
    kern = Kernel(kind, 1.3, 0.4)
    r = np.array([0.05, 0.3, 0.9, 1.7])
    h = 1e-6
    fd = (oracle.kappa(r + h, kern) - oracle.kappa(r - h, kern)) / (2 * h)
    assert np.allclose(oracle.dkappa_dr(r, kern), fd, rtol=1e-7, atol=1e-10)


def test_cov_grad_x_is_the_gradient_and_zero_on_coincident_points():
    kern = Kernel(M52, 1.0, 0.3)
    rng = np.random.default_rng(0)
    xa, xb = rng.random((4, 3)), rng.random((5, 3))
    g = oracle.cov_grad_x(xa, xb, kern)
    h = 1e-6
    for p in range(4):
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (oracle.cov_matrix(xa[p] + e, xb, kern) - oracle.cov_matrix(xa[p] - e, xb, kern)) / (2 * h)
            assert np.allclose(g[p, :, c], fd[0], rtol=1e-7, atol=1e-10)
    assert np.all(oracle.cov_grad_x(xa, xa, kern)[np.arange(4), np.arange(4)] == 0.0)


def case(seed, n=90, k=6, n0=9, d=3):
    rng = np.random.default_rng(seed)
    return oracle.build_graph(rng.random((n, d)), k, n0), rng.standard_normal(n), rng.standard_normal(n)


def moved(gr, xs):
    return dataclasses.replace(gr, xs=xs)


def directional_fd(loss, gr, delta, h=1e-6):
    return (loss(moved(gr, gr.xs + h * delta)) - loss(moved(gr, gr.xs - h * delta))) / (2 * h)


@pytest.mark.parametrize("kind,nugget", [(M32, 0.0), (SE, 1e-3), (EXP, 0.0), (M52, 1e-4)])
def test_forward_loss_x_gradient_central_difference(kind, nugget):
    gr, xi, y = case(1)
    kern = Kernel(kind, 1.1, 0.3, nugget)
    s2 = 0.05

    def loss(g):
        fac = oracle.factor(g, kern)
        v = oracle.forward(g, fac, xi)
        return 0.5 * np.sum((v - y) ** 2) / s2 + oracle.logdet(fac)

    fac = oracle.factor(gr, kern)
    v = oracle.forward(gr, fac, xi)
    _, _, gx = oracle.forward_vjp(gr, fac, kern, xi, v, (v - y) / s2, ld_bar=1.0, with_x=True)
    rng = np.random.default_rng(2)
    for _ in range(3):
        delta = rng.standard_normal(gr.xs.shape)
        fd = directional_fd(loss, gr, delta)
        assert np.sum(gx * delta) == pytest.approx(fd, rel=2e-6, abs=1e-6)
    for p, c in ((0, 0), (5, 2), (9, 1), (40, 0), (89, 2)):          # single coordinates, dense and sparse
        delta = np.zeros_like(gr.xs)
        delta[p, c] = 1.0
        assert gx[p, c] == pytest.approx(directional_fd(loss, gr, delta), rel=2e-6, abs=1e-6)


@pytest.mark.parametrize("kind", [M32, SE])
def test_inverse_loss_x_gradient_central_difference(kind):
    gr, v_in, xbar = case(3)
    kern = Kernel(kind, 0.9, 0.35, 1e-4)

    def loss(g):
        fac = oracle.factor(g, kern)
        return np.sum(xbar * oracle.inverse(g, fac, v_in))

    fac = oracle.factor(gr, kern)
    xi = oracle.inverse(gr, fac, v_in)
    _, _, gx = oracle.inverse_vjp(gr, fac, kern, v_in, xi, xbar, with_x=True)
    rng = np.random.default_rng(4)
    for _ in range(3):
        delta = rng.standard_normal(gr.xs.shape)
        assert np.sum(gx * delta) == pytest.approx(directional_fd(loss, gr, delta), rel=2e-6, abs=1e-6)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_logdet_x_gradient_central_difference(d):
    gr, _, _ = case(5, n=70, k=5, n0=4, d=d)
    kern = Kernel(M52, 1.0, 0.3, 1e-5)
    fac = oracle.factor(gr, kern)
    _, gx = oracle.logdet_vjp(gr, fac, kern, ld_bar=1.0, with_x=True)
    loss = lambda g: oracle.logdet(oracle.factor(g, kern))
    rng = np.random.default_rng(6)
    delta = rng.standard_normal(gr.xs.shape)
    assert np.sum(gx * delta) == pytest.approx(directional_fd(loss, gr, delta), rel=2e-6, abs=1e-7)


@pytest.mark.parametrize("n0", [1, 17])
def test_logdet_x_gradient_exact_limit_dense_closed_form(n0):
    """k = N - 1: the approximation is exact, so the gradient of its logdet
    is the dense one, 2 sum_q (K^-1)_pq dK_pq/dx_p, with K in slot order."""
    n = 40
    rng = np.random.default_rng(7)
    gr = oracle.build_graph(rng.random((n, 3)), n - 1, n0)
    kern = Kernel(M32, 1.0, 0.4, 1e-3)
    fac = oracle.factor(gr, kern)
    _, gx = oracle.logdet_vjp(gr, fac, kern, ld_bar=1.0, with_x=True)
    kmat = oracle.cov_matrix(gr.xs, gr.xs, kern, same=True)
    g = oracle.cov_grad_x(gr.xs, gr.xs, kern)
    dense = 2.0 * np.einsum("pq,pqc->pc", np.linalg.inv(kmat), g)
    assert np.allclose(gx, dense, rtol=1e-8, atol=1e-9 * np.abs(dense).max())
