"""vecchia_backward_noalloc (scratch in the library's static device array)
against vecchia_backward (caller scratch): the same derivatives, through the
C ABI, on two calls in a row with the second on a smaller input."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams, _lib

pytestmark = pytest.mark.gpu

TOL = {FP64: 1e-10, FP32: 1e-4}


def rel(a, b):
    a, b = a.double().cpu(), b.double().cpu()
    return float((a - b).abs().max() / max(b.abs().max().item(), 1e-300))


def backward_both(n, k, kind, precision, seed):
    """Factor + forward on a uniform cloud, then both entry points with every
    input (v_bar, xi_bar_in, logdet_bar) set; returns their outputs."""
    x = workloads.as_fp32_exact(workloads.uniform(n, seed))
    g = Graph(x, k, 64)
    dg = g.to_device(precision, "cuda:0", with_children=True)
    kern = KernelParams(kind, 1.2, 0.1, 1e-6 if kind == 2 else 0.0)
    fac = Factor(dg, kern)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    xi = torch.randn(n, dtype=dg.dtype, device="cuda", generator=gen)
    vbar = torch.randn(n, dtype=dg.dtype, device="cuda", generator=gen)
    xbar_in = torch.randn(n, dtype=dg.dtype, device="cuda", generator=gen)
    v = fac.forward(xi)
    ref_xb, ref_vb, ref_th = fac.backward(xi, v, v_bar=vbar, xi_bar_in=xbar_in, logdet_bar=0.7)
    lib = _lib.load()
    xb = torch.full_like(xi, float("nan"))
    vb = torch.full_like(xi, float("nan"))
    th = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    kc = kern.to_c()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.vecchia_backward_noalloc(ctypes.byref(fac.view), ctypes.byref(kc), ptr(xi), ptr(v), ptr(vbar),
                                      ptr(xbar_in), 0.7, ptr(xb), ptr(vb), ptr(th), stream)
    _lib.check(rc, "vecchia_backward_noalloc")
    torch.cuda.synchronize()
    return (ref_xb, ref_vb, ref_th), (xb, vb, th)


def test_noalloc_matches_backward_on_two_calls_the_second_smaller():
    cases = [(40000, 16, 1, FP32, 3), (9000, 32, 2, FP64, 4)]      # second call: smaller input
    for n, k, kind, precision, seed in cases:
        print("case n=%d k=%d kind=%d precision=%d" % (n, k, kind, precision), flush=True)
        ref, got = backward_both(n, k, kind, precision, seed)
        tol = TOL[precision]
        for name, a, b in zip(("xi_bar", "v_bar_out", "theta_bar"), got, ref):
            assert torch.isfinite(a).all(), name
            err = rel(a, b)
            print(name, err, "identical" if torch.equal(a, b) else "", flush=True)
            assert err <= tol, (name, err)


def test_noalloc_rejects_views_beyond_its_buffer():
    lib = _lib.load()
    cap = ctypes.c_size_t()
    assert lib.vecchia_backward_noalloc_max_bytes(ctypes.byref(cap)) == 0 and cap.value == 64 << 20
    n, n0 = (cap.value // 8) + 4096, 128
    lp = np.array([0, n0, n], np.int32)
    v = _lib.ViewStruct()
    v.n, v.k, v.kp, v.n0, v.n_levels, v.precision = n, 8, 8, n0, 1, FP64
    v.x = v.nbr = v.workspace = v.child_ptr = v.child = 256       # never dereferenced: rejected on the host
    v.level_ptr = lp.ctypes.data
    v.workspace_bytes = 1 << 40
    kc = _lib.KernelStruct(1, 1.0, 0.1, 0.0)
    rc = lib.vecchia_backward_noalloc(ctypes.byref(v), ctypes.byref(kc), ctypes.c_void_p(256), ctypes.c_void_p(512),
                                      ctypes.c_void_p(768), None, 0.0, ctypes.c_void_p(1024), None,
                                      ctypes.c_void_p(2048), None)
    assert rc == _lib.ENOMEM
    assert b"static buffer" in lib.vecchia_last_error()
