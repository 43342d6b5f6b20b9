"""Pins of the oracle's forward-mode derivatives (oracle/tangent.py): central
finite differences of the oracle's own forward and logdet, and the pairing
with the reverse mode of oracle/adjoint.py (itself pinned by finite
differences): <v_bar, J theta_dot> = <J^T v_bar, theta_dot>."""
import numpy as np
import pytest

import oracle
from oracle import Kernel, EXP, M32, SE, M52


def setup(kind, k, n0, seed, nugget=0.0):
    rng = np.random.default_rng(seed)
    x = rng.random((220, 3))
    kern = Kernel(kind, 1.2, 0.25, nugget)
    og = oracle.build_graph(x, k, n0)
    return og, kern, rng.standard_normal(220), rng.standard_normal(220)


def fwd(og, kern, xi):
    f = oracle.factor(og, kern)
    return oracle.forward(og, f, xi), oracle.logdet(f)


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
def test_theta_tangent_central_difference(kind):
    og, kern, xi, _ = setup(kind, 8, 16, 3 + kind, 1e-4 if kind == SE else 0.0)
    fac = oracle.factor(og, kern)
    h = 1e-5
    for td in ((1.0, 0.0), (0.0, 1.0), (0.3, -0.7)):
        vd, ldd = oracle.forward_jvp(og, fac, kern, xi, np.zeros_like(xi), td)
        kp = Kernel(kind, kern.sigma + h * td[0], kern.ell + h * td[1], kern.nugget)
        km = Kernel(kind, kern.sigma - h * td[0], kern.ell - h * td[1], kern.nugget)
        (vp, lp), (vm, lm) = fwd(og, kp, xi), fwd(og, km, xi)
        np.testing.assert_allclose(vd, (vp - vm) / (2 * h), rtol=1e-5, atol=1e-6 * np.abs(vd).max())
        assert abs(ldd - (lp - lm) / (2 * h)) <= 1e-6 * max(1.0, abs(ldd))


@pytest.mark.parametrize("kind", [M32, SE])
def test_tangent_pairs_with_the_reverse_mode(kind):
    og, kern, xi, vbar = setup(kind, 12, 8, 30 + kind, 1e-4 if kind == SE else 0.0)
    fac = oracle.factor(og, kern)
    v = oracle.forward(og, fac, xi)
    xi_bar, theta_bar = oracle.forward_vjp(og, fac, kern, xi, v, vbar, ld_bar=0.0)
    _, theta_bar_ld = oracle.forward_vjp(og, fac, kern, xi, v, np.zeros_like(vbar), ld_bar=1.0)
    rng = np.random.default_rng(7)
    for _ in range(3):
        td = rng.standard_normal(2)
        xd = rng.standard_normal(len(xi))
        vd, ldd = oracle.forward_jvp(og, fac, kern, xi, xd, td)
        lhs = vbar @ vd
        rhs = theta_bar @ td + xi_bar @ xd
        assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + abs(rhs) + 1.0), (lhs, rhs)
        assert abs(ldd - theta_bar_ld @ td) <= 1e-10 * max(1.0, abs(ldd))


def test_xi_tangent_is_the_forward_map():
    og, kern, xi, xd = setup(M32, 8, 16, 5)
    fac = oracle.factor(og, kern)
    vd, ldd = oracle.forward_jvp(og, fac, kern, xi, xd, (0.0, 0.0))
    np.testing.assert_allclose(vd, oracle.forward(og, fac, xd), rtol=1e-13, atol=1e-13)
    assert ldd == 0.0
