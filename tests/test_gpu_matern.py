"""General Matern kernel (kind MATERN, any nu in [1/4, 8]) on the FP64 path,
through the C ABI, against the FP64 oracle (oracle.kappa with
scipy.special.kv, pinned in tests/test_oracle_covariance.py by the closed
forms at nu = 1/2, 3/2, 5/2 and by quadrature of K_nu's integral
representation elsewhere), at the FP64 bar 1e-10: coefficients, forward,
inverse, round trip and logdet, plus the oracle's level operations on the
GPU's own factor.  The points are uniform with ell = 0.1 (cond(K_cc) at most
~7e3 over these nu and k), so no metric is conditioning-limited.  k = 64
factors in double for both storage precisions.  At
nu = 3/2 the general evaluation reproduces the closed-form kind on the GPU;
the entry points without a general-nu evaluation refuse the kernel."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import Kernel, M32, MATERN
from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams, VecchiaError
from gpu_helpers import Run, b_backward_error, oracle_run, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.mark.parametrize("nu", [0.3, 0.8, 1.7, 3.2, 6.5])
@pytest.mark.parametrize("k", [8, 16, 32])
def test_general_matern_fp64_against_oracle(nu, k):
    n = 1200 + 5 * k                                   # ragged last tile
    x = workloads.uniform(n, 60 + k)
    xi_in = workloads.white_noise(n, 160 + k)
    kern = Kernel(MATERN, 1.1, 0.1, 1e-8, nu=nu)
    run = Run(x, k, 64, kern, FP64, xi_in)
    ref = oracle_run(x, k, 64, kern, xi_in)
    fac, og = ref["fac"], ref["graph"]
    b, s = run.coefficients_by_slot()
    v_gpu = run.slot_order(run.v.cpu().numpy())
    v_in = run.storage_rounded(ref["v"])
    xi_inv = run.slot_order(run.fac.inverse(torch.from_numpy(v_in[run.g.slot]).to(run.dtype).cuda()).cpu().numpy())
    state = run.oracle_state()
    errs = {
        "b": rel_err(b, fac.b),
        "sigma": rel_err(s, fac.sigma),
        "v": rel_err(v_gpu, ref["v"]),
        "xi_roundtrip": rel_err(run.slot_order(run.xi_back.cpu().numpy()), ref["xi"]),
        "xi_inverse": rel_err(xi_inv, oracle.inverse(og, fac, v_in)),
        "logdet": abs(run.ld.item() - ref["logdet"]) / abs(ref["logdet"]),
        "state_v": rel_err(v_gpu, oracle.forward(og, state, ref["xi"])),
        "state_logdet": abs(run.ld.item() - oracle.logdet(state)) / abs(oracle.logdet(state)),
    }
    print("matern nu", nu, "k", k, errs, flush=True)
    assert run.fac.counts()[0] == 0
    assert b_backward_error(og, kern, b) <= 1e-12
    for name, e in errs.items():
        assert e <= TOL, (name, e)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_general_matern_width_64(precision):
    """k = 64 factors in double for both storage precisions (one point per
    wave); FP32 storage of b, sigma and v is judged at the FP32 bar 1e-4."""
    n = 1500
    x = workloads.uniform(n, 90)
    if precision == FP32:
        x = workloads.as_fp32_exact(x)
    xi_in = workloads.white_noise(n, 190)
    kern = Kernel(MATERN, 1.0, 0.1, 1e-8, nu=2.2)
    run = Run(x, 64, 128, kern, precision, xi_in)
    ref = oracle_run(x, 64, 128, kern, xi_in)
    b, s = run.coefficients_by_slot()
    tol = TOL if precision == FP64 else 1e-4
    errs = {"b": rel_err(b, ref["fac"].b), "sigma": rel_err(s, ref["fac"].sigma),
            "v": rel_err(run.slot_order(run.v.cpu().numpy()), ref["v"]),
            "logdet": abs(run.ld.item() - ref["logdet"]) / abs(ref["logdet"])}
    print("matern k64", precision, errs, flush=True)
    assert run.fac.counts()[0] == 0
    for name, e in errs.items():
        assert e <= tol, (name, e)


@pytest.mark.parametrize("k", [8, 32])
def test_general_matern_at_three_halves_matches_closed_form_kind(k):
    n = 900
    x = workloads.uniform(n, 70 + k)
    xi = workloads.white_noise(n, 170 + k)
    gen = Run(x, k, 64, Kernel(MATERN, 1.0, 0.1, 0.0, nu=1.5), FP64, xi)
    closed = Run(x, k, 64, Kernel(M32, 1.0, 0.1, 0.0), FP64, xi)
    bg, sg = gen.coefficients_by_slot()
    bc, sc = closed.coefficients_by_slot()
    assert rel_err(bg, bc) <= 1e-11
    assert rel_err(sg, sc) <= 1e-11
    assert rel_err(gen.v.cpu().numpy(), closed.v.cpu().numpy()) <= 1e-11
    assert abs(gen.ld.item() - closed.ld.item()) <= 1e-11 * abs(closed.ld.item())


def test_general_matern_is_refused_where_it_is_not_built():
    n = 600
    x = workloads.as_fp32_exact(workloads.uniform(n, 80))
    kp = KernelParams(MATERN, 1.0, 0.1, 0.0, 1.3)
    g = Graph(x, 16, 64)
    with pytest.raises(VecchiaError) as ex:                  # FP32 path at k <= 32
        Factor(g.to_device(FP32, "cuda:0"), kp)
    assert ex.value.code == -4
    with pytest.raises(VecchiaError) as ex:                  # nu outside [1/4, 8]
        Factor(g.to_device(FP64, "cuda:0"), KernelParams(MATERN, 1.0, 0.1, 0.0, 9.0))
    assert ex.value.code == -1
    dg = g.to_device(FP64, "cuda:0", with_children=True)
    fac = Factor(dg, kp)
    xi = torch.from_numpy(g.to_storage(workloads.white_noise(n, 81))).cuda()
    v = fac.forward(xi)
    for call in (lambda: fac.backward(xi, v, logdet_bar=1.0),
                 lambda: fac.backward_x(xi, v, logdet_bar=1.0),
                 lambda: fac.jvp(xi, v, sigma_dot=1.0)):
        with pytest.raises(VecchiaError) as ex:
            call()
        assert ex.value.code == -4
