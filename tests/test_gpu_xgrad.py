"""HIP coordinate cotangent (vecchia_backward_x) against the oracle's
x_grad (oracle/adjoint.py, pinned by central differences and by the dense
closed form in tests/test_oracle_xgrad.py), at a fixed graph.

x_bar comes back in storage order, N x 3; the oracle's is in slot order,
N x d.  Tolerances, max-norm relative: FP64 path 1e-9 (the cotangent runs
through K_cc^-1 as the theta gradient does, whose bar is 1e-9); FP32 path
1e-4 (the float-stored b, sigma and v enter every term)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import Kernel, EXP, M32, SE, M52
from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams

pytestmark = pytest.mark.gpu


class Case:
    def __init__(self, n, k, n0, kern, precision, seed, d=3):
        self.x = workloads.uniform(n, seed)[:, :d]
        if precision == FP32:
            self.x = workloads.as_fp32_exact(self.x)
        self.kern, self.d = kern, d
        self.g = Graph(self.x, k, n0)
        self.dg = self.g.to_device(precision, "cuda:0", with_children=True)
        self.fac = Factor(self.dg, KernelParams(kern.kind, kern.sigma, kern.ell, kern.nugget))
        self.dt = self.dg.dtype
        self.og = oracle.build_graph(self.x, k, n0)
        self.of = oracle.factor(self.og, kern)
        self.rng = np.random.default_rng(seed + 77)

    def dev(self, input_order):
        return torch.from_numpy(self.g.to_storage(input_order)).to(self.dt).cuda()

    def ora(self, input_order):
        return np.asarray(input_order)[self.og.perm]

    def to_slots(self, xbar_storage):
        """(N, 3) storage order -> (N, d) slot order."""
        out = np.empty((self.g.n, 3))
        out[self.g.slot] = xbar_storage.cpu().numpy()
        assert np.all(out[:, self.d:] == 0.0)
        return out[:, :self.d]


def err(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
@pytest.mark.parametrize("k", [8, 16, 32])
def test_forward_loss_x_gradient_fp64(kind, k):
    c = Case(700 + 5 * k, k, 40, Kernel(kind, 1.1, 0.2, 1e-5 if kind == SE else 0.0), FP64, 400 + k + kind)
    xi = c.rng.standard_normal(c.g.n)
    vbar = c.rng.standard_normal(c.g.n)
    v = c.fac.forward(c.dev(xi))
    gx = c.fac.backward_x(c.dev(xi), v, v_bar=c.dev(vbar), logdet_bar=0.6)
    v_o = oracle.forward(c.og, c.of, c.ora(xi))
    _, _, gx_o = oracle.forward_vjp(c.og, c.of, c.kern, c.ora(xi), v_o, c.ora(vbar), ld_bar=0.6, with_x=True)
    e = err(c.to_slots(gx), gx_o)
    print("forward x_bar", kind, k, e, flush=True)
    assert e <= 1e-9


@pytest.mark.parametrize("kind", [M32, SE])
def test_inverse_loss_x_gradient_fp64(kind):
    c = Case(900, 16, 64, Kernel(kind, 0.9, 0.25, 1e-5 if kind == SE else 0.0), FP64, 500 + kind)
    v_in = c.rng.standard_normal(c.g.n)
    xibar = c.rng.standard_normal(c.g.n)
    v = c.dev(v_in)
    xi = c.fac.inverse(v)
    gx = c.fac.backward_x(xi, v, xi_bar_in=c.dev(xibar))
    xi_o = oracle.inverse(c.og, c.of, c.ora(v_in))
    _, _, gx_o = oracle.inverse_vjp(c.og, c.of, c.kern, c.ora(v_in), xi_o, c.ora(xibar), with_x=True)
    e = err(c.to_slots(gx), gx_o)
    print("inverse x_bar", kind, e, flush=True)
    assert e <= 1e-9


@pytest.mark.parametrize("d", [1, 2, 3])
def test_logdet_x_gradient_fp64_and_dense_limit(d):
    """logdet alone (every dimension count), and k = N - 1 where it is the
    dense 2 sum_q (K^-1)_pq dK_pq/dx_p."""
    c = Case(600, 16, 32, Kernel(M52, 1.0, 0.3, 1e-5), FP64, 600 + d, d=d)
    xi = np.zeros(c.g.n)
    v = c.fac.forward(c.dev(xi))
    gx = c.fac.backward_x(c.dev(xi), v, logdet_bar=1.0)
    _, gx_o = oracle.logdet_vjp(c.og, c.of, c.kern, ld_bar=1.0, with_x=True)
    assert err(c.to_slots(gx), gx_o) <= 1e-9
    n = 33
    e = Case(n, 32, 1, Kernel(M32, 1.0, 0.5, 1e-3), FP64, 700 + d, d=d)
    v = e.fac.forward(e.dev(np.zeros(n)))
    gx = e.to_slots(e.fac.backward_x(e.dev(np.zeros(n)), v, logdet_bar=1.0))
    kmat = oracle.cov_matrix(e.og.xs, e.og.xs, e.kern, same=True)
    dense = 2.0 * np.einsum("pq,pqc->pc", np.linalg.inv(kmat), oracle.cov_grad_x(e.og.xs, e.og.xs, e.kern))
    assert err(gx, dense) <= 1e-8


@pytest.mark.parametrize("kind", [M32, SE])
def test_forward_loss_x_gradient_fp32(kind):
    c = Case(1500, 16, 64, Kernel(kind, 1.0, 0.15, 1e-4 if kind == SE else 0.0), FP32, 800 + kind)
    xi = c.rng.standard_normal(c.g.n)
    vbar = c.rng.standard_normal(c.g.n)
    v = c.fac.forward(c.dev(xi))
    gx = c.fac.backward_x(c.dev(xi), v, v_bar=c.dev(vbar), logdet_bar=1.0)
    v_o = oracle.forward(c.og, c.of, c.ora(xi))
    _, _, gx_o = oracle.forward_vjp(c.og, c.of, c.kern, c.ora(xi), v_o, c.ora(vbar), ld_bar=1.0, with_x=True)
    e = err(c.to_slots(gx), gx_o)
    print("forward x_bar fp32", kind, e, flush=True)
    assert e <= 1e-4


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
def test_width_64_forward_and_logdet_x_gradient_fp64(kind):
    """k = 64 runs on the one-point-per-wave kernel (lane = row)."""
    c = Case(700, 64, 70, Kernel(kind, 1.0, 0.3, 1e-4 if kind == SE else 0.0), FP64, 900 + kind)
    xi = c.rng.standard_normal(c.g.n)
    vbar = c.rng.standard_normal(c.g.n)
    v = c.fac.forward(c.dev(xi))
    gx = c.fac.backward_x(c.dev(xi), v, v_bar=c.dev(vbar), logdet_bar=0.8)
    v_o = oracle.forward(c.og, c.of, c.ora(xi))
    _, _, gx_o = oracle.forward_vjp(c.og, c.of, c.kern, c.ora(xi), v_o, c.ora(vbar), ld_bar=0.8, with_x=True)
    e = err(c.to_slots(gx), gx_o)
    print("forward x_bar k64", kind, e, flush=True)
    assert e <= 1e-9


def test_width_64_inverse_x_gradient_fp32():
    c = Case(900, 64, 80, Kernel(M32, 1.0, 0.2), FP32, 950)
    v_in = c.rng.standard_normal(c.g.n)
    xibar = c.rng.standard_normal(c.g.n)
    v = c.dev(v_in)
    xi = c.fac.inverse(v)
    gx = c.fac.backward_x(xi, v, xi_bar_in=c.dev(xibar))
    xi_o = oracle.inverse(c.og, c.of, c.ora(v_in))
    _, _, gx_o = oracle.inverse_vjp(c.og, c.of, c.kern, c.ora(v_in), xi_o, c.ora(xibar), with_x=True)
    e = err(c.to_slots(gx), gx_o)
    print("inverse x_bar k64 fp32", e, flush=True)
    assert e <= 1e-4
