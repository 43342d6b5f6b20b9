"""HIP adjoint (vecchia_backward) against the oracle's reverse-mode
derivatives, finite differences of the oracle, and the adjoint identity.

Tolerances: FP64 path 1e-10 on the white-noise / field cotangents (max-norm
relative) and 1e-9 on theta (relative); FP32 path 1e-4."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import Kernel, EXP, M32, SE, M52
from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams
from paper_2606_11402_amd import autograd as vag
from gpu_helpers import rel_err

pytestmark = pytest.mark.gpu


class Case:
    def __init__(self, n, k, n0, kern, precision, seed, dist="uniform"):
        gen = {"uniform": workloads.uniform, "radial": workloads.radial}[dist]
        self.x = gen(n, seed)
        if precision == FP32:
            self.x = workloads.as_fp32_exact(self.x)
        self.kern = kern
        self.g = Graph(self.x, k, n0)
        self.dg = self.g.to_device(precision, "cuda:0", with_children=True)
        self.fac = Factor(self.dg, KernelParams(kern.kind, kern.sigma, kern.ell, kern.nugget))
        self.dt = self.dg.dtype
        self.og = oracle.build_graph(self.x, k, n0)
        self.of = oracle.factor(self.og, kern)
        self.rng = np.random.default_rng(seed + 1000)

    def dev(self, input_order):
        return torch.from_numpy(self.g.to_storage(input_order)).to(self.dt).cuda()

    def slot(self, storage_tensor):
        out = np.empty(self.g.n)
        out[self.g.slot] = storage_tensor.double().cpu().numpy()
        return out

    def ora(self, input_order):
        return np.asarray(input_order)[self.og.perm]


def theta_err(a, ref):
    return float(np.max(np.abs(np.asarray(a) - ref) / np.abs(ref)))


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
@pytest.mark.parametrize("k", [8, 16, 32, 64])
def test_forward_vjp_fp64(kind, k):
    c = Case(900 + 3 * k, k, 48, Kernel(kind, 1.2, 0.2, 1e-5 if kind == SE else 0.0), FP64, 200 + k)
    xi = c.rng.standard_normal(c.g.n)
    vbar = c.rng.standard_normal(c.g.n)
    v = c.fac.forward(c.dev(xi))
    xi_bar, _, theta = c.fac.backward(c.dev(xi), v, v_bar=c.dev(vbar), logdet_bar=0.7)
    v_o = oracle.forward(c.og, c.of, c.ora(xi))
    xb_o, th_o = oracle.forward_vjp(c.og, c.of, c.kern, c.ora(xi), v_o, c.ora(vbar), ld_bar=0.7)
    e_xi = rel_err(c.slot(xi_bar), xb_o)
    e_th = theta_err(theta.cpu().numpy(), th_o)
    print("forward vjp", kind, k, e_xi, e_th, theta.cpu().numpy(), th_o, flush=True)
    assert e_xi <= 1e-10 and e_th <= 1e-9


@pytest.mark.parametrize("kind", [EXP, M32, SE])
def test_inverse_vjp_fp64(kind):
    c = Case(1000, 16, 64, Kernel(kind, 0.9, 0.25, 1e-5 if kind == SE else 0.0), FP64, 300 + kind)
    v_in = c.rng.standard_normal(c.g.n)
    xibar = c.rng.standard_normal(c.g.n)
    v = c.dev(v_in)
    xi = c.fac.inverse(v)
    _, v_bar, theta = c.fac.backward(xi, v, xi_bar_in=c.dev(xibar))
    xi_o = oracle.inverse(c.og, c.of, c.ora(v_in))
    vb_o, th_o = oracle.inverse_vjp(c.og, c.of, c.kern, c.ora(v_in), xi_o, c.ora(xibar))
    e_v = rel_err(c.slot(v_bar), vb_o)
    e_th = theta_err(theta.cpu().numpy(), th_o)
    print("inverse vjp", kind, e_v, e_th, flush=True)
    assert e_v <= 1e-10 and e_th <= 1e-9


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_logdet_vjp(precision):
    c = Case(1500, 8, 128, Kernel(M32, 1.4, 0.1), precision, 400)
    z = torch.zeros(c.g.n, dtype=c.dt, device="cuda")
    _, _, theta = c.fac.backward(z, z, logdet_bar=1.0)
    th_o = oracle.logdet_vjp(c.og, c.of, c.kern, 1.0)
    e = theta_err(theta.cpu().numpy(), th_o)
    print("logdet vjp", precision, e, flush=True)
    assert e <= (1e-9 if precision == FP64 else 1e-4)
    assert theta[0].item() == pytest.approx(2 * c.g.n / 1.4, rel=1e-9 if precision == FP64 else 1e-4)


def test_adjoint_identity_large():
    """<vbar, F xi> = <F^T vbar, xi> at 2^18 points (FP64)."""
    n = 1 << 18
    x = workloads.uniform(n, 500)
    g = Graph(x, 16, 128)
    dg = g.to_device(FP64, "cuda:0", with_children=True)
    fac = Factor(dg, KernelParams(M32, 1.0, 0.05))
    gen = torch.Generator(device="cuda").manual_seed(5)
    xi = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
    vbar = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
    v = fac.forward(xi)
    xi_bar, _, _ = fac.backward(xi, v, v_bar=vbar)
    lhs = torch.dot(vbar, v).item()
    rhs = torch.dot(xi_bar, xi).item()
    assert abs(lhs - rhs) <= 1e-11 * (torch.linalg.norm(vbar) * torch.linalg.norm(v)).item()


C4_FP32_THETA_CAP = 1e-3   # regression cap of the FP32 end-to-end theta error; it meets 1e-4 today (the policy factors this cloud in double)


def c4_loss_oracle(og, kern, xi_slot, y_slot, s2):
    f = oracle.factor(og, kern)
    v = oracle.forward(og, f, xi_slot)
    return 0.5 * np.sum((v - y_slot) ** 2) / s2 + oracle.logdet(f)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_workload4_loss_gradients(precision):
    """Workload 4's loss 1/2 |v - y|^2 / s^2 + logdet (s = 0.1), radial cloud,
    Matern-3/2, k = 16, at N = 2^13: autograd gradients in xi, sigma, ell
    against the oracle's gradient and central differences (h = 1e-4) of the
    oracle's loss."""
    w = workloads.WORKLOADS[4]
    n = 1 << 13
    kern = Kernel(w.kind, w.sigma, w.ell, w.nugget)
    x = w.points(n)
    gr = Graph(x, w.k, 128)
    gp = vag.GaussianProcess(gr, w.kind, w.nugget, precision, "cuda:0")
    dt = gp.dtype
    xi_in, y_in = w.xi(n), w.data(n)
    s2 = 0.1 ** 2
    xi = torch.from_numpy(gr.to_storage(xi_in)).to(dt).cuda().requires_grad_(True)
    y = torch.from_numpy(gr.to_storage(y_in)).to(dt).cuda()
    sigma = torch.tensor(w.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    ell = torch.tensor(w.ell, dtype=torch.float64, device="cuda", requires_grad=True)
    v = vag.forward(gp, xi, sigma, ell)
    loss = 0.5 * torch.sum((v.double() - y.double()) ** 2) / s2 + vag.logdet(gp, sigma, ell)
    loss.backward()

    og = oracle.build_graph(x, w.k, 128)
    of = oracle.factor(og, kern)
    xs, ys = xi_in[og.perm], y_in[og.perm]
    vo = oracle.forward(og, of, xs)
    gxi_o, gth_o = oracle.forward_vjp(og, of, kern, xs, vo, (vo - ys) / s2, ld_bar=1.0)
    gxi = np.empty(n)
    gxi[gr.slot] = xi.grad.double().cpu().numpy()
    h = 1e-4
    fd = []
    for t in range(2):
        kp = Kernel(w.kind, w.sigma + h * (t == 0), w.ell + h * (t == 1), w.nugget)
        km = Kernel(w.kind, w.sigma - h * (t == 0), w.ell - h * (t == 1), w.nugget)
        fd.append((c4_loss_oracle(og, kp, xs, ys, s2) - c4_loss_oracle(og, km, xs, ys, s2)) / (2 * h))
    got = np.array([sigma.grad.item(), ell.grad.item()])
    errs = {"xi": rel_err(gxi, gxi_o), "theta_vs_oracle": theta_err(got, gth_o),
            "theta_vs_fd": theta_err(got, np.array(fd)), "oracle_vs_fd": theta_err(gth_o, np.array(fd))}
    # the oracle's gradient at the GPU's own forward state (its b, sigma and
    # v): isolates the adjoint from the error that the storage precision
    # leaves in that state
    fac = gp.factor(w.sigma, w.ell)
    b_dev, s_dev = fac.coefficients()
    b_dev = gr.to_row_order(b_dev)
    rows = gr.slot[128:] - 128
    b_slot = np.empty((gr.ns, gr.k))
    s_slot = np.empty(gr.ns)
    b_slot[rows], s_slot[rows] = b_dev, s_dev
    state = oracle.Factor(of.L0, b_slot, s_slot)
    v_dev = np.empty(n)
    v_dev[gr.slot] = v.detach().double().cpu().numpy()
    _, gth_state = oracle.forward_vjp(og, state, kern, xs, v_dev, (v_dev - ys) / s2, ld_bar=1.0)
    errs["theta_vs_oracle_same_state"] = theta_err(got, gth_state)
    errs["oracle_state_vs_oracle"] = theta_err(gth_state, gth_o)
    print("workload4 gradients", precision, errs, got, gth_o, gth_state, fd, flush=True)
    tol = 1e-10 if precision == FP64 else 1e-4
    assert errs["oracle_vs_fd"] <= 1e-5          # the oracle's own pin at this step size
    assert errs["xi"] <= tol and errs["theta_vs_oracle_same_state"] <= max(tol, 1e-9)
    if precision == FP64:
        assert errs["theta_vs_fd"] <= 1e-5 and errs["theta_vs_oracle"] <= 1e-9
    elif errs["theta_vs_oracle"] > tol:
        # end to end, the float forward state alone moves the exact gradient
        # by oracle_state_vs_oracle; the adjoint adds no more than tol to it.
        # Regression cap: the measured end-to-end error times ten.
        assert errs["theta_vs_oracle"] <= errs["oracle_state_vs_oracle"] + tol
        assert errs["theta_vs_oracle"] <= C4_FP32_THETA_CAP, errs["theta_vs_oracle"]
        pytest.xfail("FP32 theta gradient %.2e from the FP64 oracle: the float forward state (b, sigma, v) "
                     "alone accounts for %.2e; the adjoint at that state agrees to %.2e"
                     % (errs["theta_vs_oracle"], errs["oracle_state_vs_oracle"],
                        errs["theta_vs_oracle_same_state"]))
