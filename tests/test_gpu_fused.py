"""The fused on-the-fly forward (Alg. 1 as written: K_cc rebuilt and factored
per point inside the batch loop, no coefficients stored) against the FP64
oracle's forward and logdet, and against the stored-coefficient forward on
the same graph.  Bars: FP64 1e-10, FP32 storage 1e-4 (relative, as in the
other parity tests)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import Kernel, EXP, M32, SE, M52
from paper_2606_11402_amd import FP32, FP64, Factor, FusedForward, Graph, KernelParams, VecchiaError
from gpu_helpers import rel_err

pytestmark = pytest.mark.gpu

TOL = {FP64: 1e-10, FP32: 1e-4}


def run_fused(x, k, n0, kern, precision, xi_in):
    g = Graph(x, k, n0)
    dg = g.to_device(precision, "cuda:0")
    kp = KernelParams(kern.kind, kern.sigma, kern.ell, kern.nugget)
    ff = FusedForward(dg, kp)
    xi = torch.from_numpy(g.to_storage(xi_in)).to(dg.dtype).cuda()
    ld = torch.empty(1, dtype=torch.float64, device="cuda")
    v = ff(xi, logdet=ld)
    ff.status()
    torch.cuda.synchronize()
    return g, dg, kp, xi, v, ld.item()


def slot_order(g, a):
    out = np.empty_like(a)
    out[g.slot] = a
    return out


def against_oracle(x, k, n0, kern, precision, xi_in):
    g, dg, kp, xi, v, ld = run_fused(x, k, n0, kern, precision, xi_in)
    og = oracle.build_graph(x, k, n0)
    of = oracle.factor(og, kern)
    v_ref = oracle.forward(og, of, np.asarray(xi_in)[og.perm])
    ld_ref = oracle.logdet(of)
    errs = {"v": rel_err(slot_order(g, v.double().cpu().numpy()), v_ref), "logdet": abs(ld - ld_ref) / abs(ld_ref)}
    # the stored-coefficient path on the same graph and input
    fac = Factor(dg, kp)
    v_stored = fac.forward(xi)
    ld_stored = fac.logdet().item()
    errs["v_vs_stored"] = rel_err(v.double().cpu().numpy(), v_stored.double().cpu().numpy())
    errs["logdet_vs_stored"] = abs(ld - ld_stored) / abs(ld_stored)
    print("fused", precision, k, kern.kind, errs, flush=True)
    tol = TOL[precision]
    for name, e in errs.items():
        assert e <= tol, (name, e)
    return errs


@pytest.mark.parametrize("kind", [EXP, M32, SE, M52])
@pytest.mark.parametrize("k", [5, 8, 16, 32, 64])
def test_fused_forward_fp64(kind, k):
    n = 1700 + 11 * k                      # ragged last tile
    x = workloads.uniform(n, 300 + k)
    kern = Kernel(kind, 1.1, 0.15, 1e-6 if kind == SE else 0.0)
    against_oracle(x, k, 64, kern, FP64, workloads.white_noise(n, 400 + k))


@pytest.mark.parametrize("k", [8, 16, 32, 64])
def test_fused_forward_fp32_storage(k):
    n = 3000 + 13 * k
    x = workloads.as_fp32_exact(workloads.uniform(n, 310 + k))
    against_oracle(x, k, 128, Kernel(M32, 1.0, 0.1), FP32, workloads.white_noise(n, 410 + k))


def test_fused_workload1_full():
    w = workloads.WORKLOADS[1]
    against_oracle(w.points(), w.k, 128, Kernel(w.kind, w.sigma, w.ell, w.nugget), FP64, w.xi())


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_fused_radial_workload2_shape(precision):
    """Workload 2's radial cloud and Matern-3/2 at N = 2^14: the fused pass
    computes in double, so the FP32 storage path meets its bar here too."""
    w = workloads.WORKLOADS[2]
    n = 1 << 14
    against_oracle(w.points(n), w.k, 128, Kernel(w.kind, w.sigma, w.ell, w.nugget), precision, w.xi(n))


def test_fused_edge_cases():
    kern = Kernel(M32, 1.0, 0.2)
    for n, k, n0 in ((128, 8, 128), (129, 8, 128), (100, 8, 1), (70, 64, 1)):
        x = workloads.uniform(n, 500 + n)
        xi = workloads.white_noise(n, 600 + n)
        g, dg, kp, xit, v, ld = run_fused(x, k, n0, kern, FP64, xi)
        og = oracle.build_graph(x, k, n0)
        of = oracle.factor(og, kern)
        assert rel_err(slot_order(g, v.cpu().numpy()), oracle.forward(og, of, xi[og.perm])) <= 1e-10, (n, k, n0)
        assert abs(ld - oracle.logdet(of)) <= 1e-10 * abs(oracle.logdet(of)), (n, k, n0)


def test_fused_not_positive_definite_is_reported():
    x = workloads.uniform(2000, 70)
    x[1000:1040] = x[5]
    g = Graph(x, 8, 64)
    dg = g.to_device(FP64, "cuda:0")
    ff = FusedForward(dg, KernelParams(SE, 1.0, 0.1, 0.0))
    ff(torch.zeros(g.n, dtype=torch.float64, device="cuda"))
    with pytest.raises(VecchiaError) as e:
        ff.status()
    assert e.value.code == -3
