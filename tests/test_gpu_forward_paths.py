"""The forward as the library runs it (one workgroup per run of small
batches, with the run's values in LDS; one launch per larger batch) against
the forward with one launch per batch for every batch.  Both evaluate every
v_i with the same operations in the same order, so they must agree bit for
bit; the per-batch forward is itself checked against the oracle in
test_gpu_parity.py.  Sizes are chosen so that both kinds of batches occur and
that runs outgrow the LDS copy (runs whose LDS starts at position 0 and runs
whose LDS starts at their own first position, reading earlier values from
HBM); FP64 at k = 32 runs with the half-size workgroup."""
import numpy as np
import pytest
import torch

import workloads
from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams

pytestmark = pytest.mark.gpu

SMALL_BATCH = 512    # batches up to this size go to the one-workgroup run kernel


@pytest.mark.parametrize("wl,n,k,precision", [(3, 1 << 21, 32, FP32), (2, 1 << 20, 16, FP32),
                                              (1, 1 << 19, 8, FP64), (3, 1 << 21, 32, FP64)])
def test_forward_paths_match_per_batch(wl, n, k, precision):
    w = workloads.WORKLOADS[wl]
    print("forward paths: workload", wl, "n", n, "k", k, "precision", precision, flush=True)
    g = Graph(w.points(n), k, w.n0)
    sizes = np.diff(np.asarray(g.level_ptr)[1:])
    assert (sizes > SMALL_BATCH).sum() >= 2 and (sizes <= SMALL_BATCH).sum() >= 2
    dg = g.to_device(precision, "cuda:0")
    fac = Factor(dg, KernelParams(w.kind, w.sigma, w.ell, w.nugget))
    xi = torch.from_numpy(g.to_storage(w.xi(n))).to(dg.dtype).cuda()
    v_batch = fac.forward(xi, per_batch=True)
    v_flow = [fac.forward(xi) for _ in range(3)]
    fac.status()
    for v in v_flow:
        assert torch.equal(v, v_batch)
    if precision == FP64:
        xi_back = fac.inverse(v_flow[0])
        assert ((xi_back - xi).abs().max() / xi.abs().max()).item() < 1e-10


@pytest.mark.parametrize("repeats", [1, 2])
def test_forward_with_empty_batches_in_view(repeats):
    """Empty batches in level_ptr (allowed by the view) change nothing: one
    alone, or two in a row (a run made of empty batches only, no LDS)."""
    w = workloads.WORKLOADS[2]
    n, k = 1 << 19, 16
    g = Graph(w.points(n), k, w.n0)
    lp = np.asarray(g.level_ptr).copy()
    sizes = np.diff(lp[1:])
    big = int(np.argmax(sizes)) + 1       # level index of the largest batch
    # repeat one boundary: `repeats` empty batches, the following one takes the points of `big`
    lp2 = np.concatenate([lp[:big + 1]] + [lp[big:big + 1]] * (repeats - 1) + [lp[big:]]).astype(np.int32)
    dg = g.to_device(FP32, "cuda:0")
    fac = Factor(dg, KernelParams(w.kind, w.sigma, w.ell, w.nugget))
    xi = torch.from_numpy(g.to_storage(w.xi(n))).float().cuda()
    v_ref = fac.forward(xi, per_batch=True)
    fac.view.level_ptr = lp2.ctypes.data
    fac.view.n_levels = dg.n_levels + repeats
    lp_dev = torch.from_numpy(lp2).cuda()
    fac.view.level_ptr_dev = lp_dev.data_ptr()
    v = fac.forward(xi)
    fac.status()
    assert torch.equal(v, v_ref)
