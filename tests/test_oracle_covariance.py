"""Pins of oracle.covariance against library routines and finite differences."""
import numpy as np
import pytest
import scipy.special
import scipy.stats

import oracle
from oracle import Kernel, EXP, M32, SE, M52


def matern_general(r, nu, sigma, ell):
    # scipy route: sigma^2 2^(1-nu)/Gamma(nu) (sqrt(2 nu) r/ell)^nu K_nu(sqrt(2 nu) r/ell)
    z = np.sqrt(2.0 * nu) * r / ell
    return sigma ** 2 * 2.0 ** (1.0 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z)


R = np.array([1e-4, 0.003, 0.05, 0.1, 0.37, 1.0, 2.5])


def test_exp_is_matern_half():
    k = Kernel(EXP, sigma=1.3, ell=0.2)
    np.testing.assert_allclose(oracle.kappa(R, k), matern_general(R, 0.5, 1.3, 0.2), rtol=1e-12)


def test_m32_is_matern_three_halves():
    k = Kernel(M32, sigma=0.7, ell=0.05)
    np.testing.assert_allclose(oracle.kappa(R, k), matern_general(R, 1.5, 0.7, 0.05), rtol=1e-10)


def test_m52_is_matern_five_halves():
    k = Kernel(M52, sigma=1.2, ell=0.08)
    np.testing.assert_allclose(oracle.kappa(R, k), matern_general(R, 2.5, 1.2, 0.08), rtol=1e-10)
    assert oracle.kappa(0.0, k) == pytest.approx(1.44, rel=1e-15)      # kappa(0) = sigma^2


def test_se_is_scaled_normal_pdf():
    k = Kernel(SE, sigma=2.0, ell=0.3)
    ref = 4.0 * scipy.stats.norm.pdf(R, scale=0.3) * 0.3 * np.sqrt(2.0 * np.pi)
    np.testing.assert_allclose(oracle.kappa(R, k), ref, rtol=1e-13)


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
def test_derivatives_central_difference(kind):
    h = 1e-6
    k = Kernel(kind, sigma=1.1, ell=0.15)
    for name, fn in (("sigma", oracle.dkappa_dsigma), ("ell", oracle.dkappa_dell)):
        kp = Kernel(kind, sigma=k.sigma + (h if name == "sigma" else 0), ell=k.ell + (h if name == "ell" else 0))
        km = Kernel(kind, sigma=k.sigma - (h if name == "sigma" else 0), ell=k.ell - (h if name == "ell" else 0))
        fd = (oracle.kappa(R, kp) - oracle.kappa(R, km)) / (2 * h)
        np.testing.assert_allclose(fn(R, k), fd, rtol=1e-7, atol=1e-9)   # FD rounding ~ eps*kappa/h


def test_nugget_only_on_same_index():
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])   # duplicate point
    k = Kernel(EXP, 1.0, 1.0, nugget=0.5)
    m = oracle.cov_matrix(x, x, k, same=True)
    assert m[0, 0] == 1.5 and m[1, 1] == 1.5 and m[0, 1] == 1.0
    assert oracle.cov_matrix(x, x, k, deriv="sigma")[0, 0] == 2.0


# ---- kind MATERN (any nu): pinned by the closed forms at the half-integers
# and, elsewhere, by K_nu from a quadrature of its integral representation
# K_nu(a) = int_0^inf exp(-a cosh t) cosh(nu t) dt (no Bessel routine).

@pytest.mark.parametrize("nu,closed", [(0.5, EXP), (1.5, M32), (2.5, M52)])
def test_matern_general_at_half_integers_is_the_closed_form(nu, closed):
    r = np.array([0.0, 1e-6, 0.01, 0.07, 0.3, 0.9, 2.5])
    gen = oracle.kappa(r, Kernel(oracle.MATERN, 1.4, 0.35, nu=nu))
    ref = oracle.kappa(r, Kernel(closed, 1.4, 0.35))
    assert np.allclose(gen, ref, rtol=1e-13, atol=0.0)


def _k_nu_quadrature(nu, a):
    import scipy.integrate
    f = lambda t: np.exp(-a * np.cosh(t)) * np.cosh(nu * t)
    upper = np.arccosh(max(1.0, 800.0 / a)) + 1.0
    val, _ = scipy.integrate.quad(f, 0.0, upper, epsabs=0.0, epsrel=1e-13, limit=400)
    return val


@pytest.mark.parametrize("nu", [0.3, 0.8, 1.0, 2.2, 3.7, 7.5])
def test_matern_general_against_integral_representation(nu):
    kern = Kernel(oracle.MATERN, 0.9, 0.2, nu=nu)
    for r in (0.003, 0.05, 0.2, 0.6):
        a = np.sqrt(2.0 * nu) * r / kern.ell
        ref = kern.sigma ** 2 * 2.0 ** (1.0 - nu) / scipy.special.gamma(nu) * a ** nu * _k_nu_quadrature(nu, a)
        assert float(oracle.kappa(r, kern)) == pytest.approx(ref, rel=1e-10)


def test_matern_general_limit_and_monotone_decay():
    kern = Kernel(oracle.MATERN, 1.2, 0.3, nu=1.3)
    r = np.linspace(0.0, 2.0, 400)
    k = oracle.kappa(r, kern)
    assert k[0] == kern.sigma ** 2
    assert abs(k[1] - k[0]) < 1e-3 * k[0]                 # continuous at 0
    assert np.all(np.diff(k) < 0.0)
