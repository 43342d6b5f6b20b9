"""Stationary covariance kernels kappa(r) and their parameter derivatives (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2.1 works with a stationary, decaying kernel K = kappa(|x - x'|).  The
paper does not fix its form; the benchmark workloads name three, written here
with amplitude sigma (variance sigma^2), length scale ell and an absolute
nugget tau added only where the two arguments are the same point (same index):

* EXP: sigma^2 exp(-r/ell)                      (Matern nu = 1/2)
* M32: sigma^2 (1 + a) exp(-a),  a = sqrt(3) r/ell   (Matern nu = 3/2)
* SE : sigma^2 exp(-r^2 / (2 ell^2))                  (Matern nu -> infinity)
* M52: sigma^2 (1 + a + a^2/3) exp(-a),  a = sqrt(5) r/ell   (Matern nu = 5/2)

The accuracy study of Fig. 1 uses the Matern family with a smoothing
parameter nu; the half-integer members have the closed forms above, and
kind MATERN is the family at any nu (Rasmussen and Williams, Eq. 4.14):

* MATERN: sigma^2 2^(1 - nu) / Gamma(nu) a^nu K_nu(a),  a = sqrt(2 nu) r / ell,
  with K_nu the modified Bessel function of the second kind
  (scipy.special.kv) and the limit sigma^2 at r = 0.  Only its value is
  written here (no parameter or distance derivatives).

Derivatives (nugget excluded): d/dsigma = 2 kappa / sigma and
d/dell = kappa r/ell^2 (EXP), sigma^2 a^2 exp(-a)/ell (M32),
kappa r^2/ell^3 (SE), sigma^2 a^2 (1 + a) exp(-a) / (3 ell) (M52);
in the distance, d kappa/dr = -kappa/ell (EXP), -sigma^2 a exp(-a) sqrt(3)/ell
(M32), -kappa r/ell^2 (SE), -sigma^2 (a/3)(1 + a) exp(-a) sqrt(5)/ell (M52),
and in a coordinate, d kappa(|x_p - x_q|)/d x_p = kappa'(r) (x_p - x_q)/r,
taken as 0 where r = 0 (a point with itself; the nugget has no coordinate).

Pins (tests/test_oracle_covariance.py): EXP, M32 and M52 against the general
Matern form built from scipy.special.kv; SE against scipy.stats.norm.pdf;
every derivative against a central finite difference; MATERN at nu = 1/2,
3/2 and 5/2 against EXP, M32 and M52, and at other nu against K_nu from a
quadrature of its integral representation (no Bessel routine).
"""
from dataclasses import dataclass

import numpy as np
import scipy.special

EXP, M32, SE, M52, MATERN = 0, 1, 2, 3, 4


@dataclass(frozen=True)
class Kernel:
    kind: int
    sigma: float = 1.0
    ell: float = 1.0
    nugget: float = 0.0
    nu: float = 0.0          # smoothing of kind MATERN (unused by the others)


def kappa(r, kern):
    r = np.asarray(r, dtype=np.float64)
    s2 = kern.sigma * kern.sigma
    if kern.kind == EXP:
        return s2 * np.exp(-r / kern.ell)
    if kern.kind == M32:
        a = np.sqrt(3.0) * r / kern.ell
        return s2 * (1.0 + a) * np.exp(-a)
    if kern.kind == SE:
        return s2 * np.exp(-(r * r) / (2.0 * kern.ell * kern.ell))
    if kern.kind == M52:
        a = np.sqrt(5.0) * r / kern.ell
        return s2 * (1.0 + a + a * a / 3.0) * np.exp(-a)
    if kern.kind == MATERN:
        nu = float(kern.nu)
        a = np.sqrt(2.0 * nu) * r / kern.ell
        with np.errstate(invalid="ignore", divide="ignore"):
            val = s2 * 2.0 ** (1.0 - nu) / scipy.special.gamma(nu) * a ** nu * scipy.special.kv(nu, a)
        return np.where(a > 0.0, val, s2)
    raise ValueError("unknown kernel kind %r" % (kern.kind,))


def dkappa_dsigma(r, kern):
    return 2.0 * kappa(r, kern) / kern.sigma


def dkappa_dell(r, kern):
    r = np.asarray(r, dtype=np.float64)
    if kern.kind == EXP:
        return kappa(r, kern) * r / (kern.ell * kern.ell)
    if kern.kind == M32:
        a = np.sqrt(3.0) * r / kern.ell
        return kern.sigma * kern.sigma * a * a * np.exp(-a) / kern.ell
    if kern.kind == SE:
        return kappa(r, kern) * r * r / (kern.ell ** 3)
    if kern.kind == M52:
        a = np.sqrt(5.0) * r / kern.ell
        return kern.sigma * kern.sigma * a * a * (1.0 + a) * np.exp(-a) / (3.0 * kern.ell)
    raise ValueError("unknown kernel kind %r" % (kern.kind,))


def dkappa_dr(r, kern):
    r = np.asarray(r, dtype=np.float64)
    s2 = kern.sigma * kern.sigma
    if kern.kind == EXP:
        return -kappa(r, kern) / kern.ell
    if kern.kind == M32:
        a = np.sqrt(3.0) * r / kern.ell
        return -s2 * a * np.exp(-a) * np.sqrt(3.0) / kern.ell
    if kern.kind == SE:
        return -kappa(r, kern) * r / (kern.ell * kern.ell)
    if kern.kind == M52:
        a = np.sqrt(5.0) * r / kern.ell
        return -s2 * (a / 3.0) * (1.0 + a) * np.exp(-a) * np.sqrt(5.0) / kern.ell
    raise ValueError("unknown kernel kind %r" % (kern.kind,))


def cov_grad_x(xa, xb, kern):
    """g[p, q] = d kappa(|xa_p - xb_q|) / d xa_p, shape (m, n, d); the
    derivative in xb_q is -g[p, q].  Zero where the two points coincide."""
    xa = np.atleast_2d(np.asarray(xa, dtype=np.float64))
    xb = np.atleast_2d(np.asarray(xb, dtype=np.float64))
    diff = xa[:, None, :] - xb[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    scale = np.where(r > 0, dkappa_dr(r, kern) / np.where(r > 0, r, 1.0), 0.0)
    return scale[:, :, None] * diff


def pairwise_r(xa, xb):
    """Euclidean distances between the rows of xa (m, d) and xb (n, d)."""
    xa = np.atleast_2d(np.asarray(xa, dtype=np.float64))
    xb = np.atleast_2d(np.asarray(xb, dtype=np.float64))
    diff = xa[:, None, :] - xb[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


def cov_matrix(xa, xb, kern, same=False, deriv=None):
    """kappa(|xa_p - xb_q|); with same=True (xa is xb) the nugget is added on
    the diagonal.  deriv in {None, 'sigma', 'ell'} returns the derivative of
    the matrix with respect to that parameter instead (the nugget has none)."""
    r = pairwise_r(xa, xb)
    if deriv is None:
        k = kappa(r, kern)
        if same:
            k = k + kern.nugget * np.eye(k.shape[0])
        return k
    if deriv == "sigma":
        return dkappa_dsigma(r, kern)
    if deriv == "ell":
        return dkappa_dell(r, kern)
    raise ValueError(deriv)
