"""The order/accuracy study on the GPU factor (paper_2606_11402_amd/study.py):
the KL divergence of the Vecchia approximation from the exact GP computed
from the HIP factor (b, sigma, L0, logdet) against the textbook dense KL of
the oracle's factor; zero in the exact limit (Sec. 2.1); non-negative and
non-increasing in k."""
import numpy as np
import pytest

import oracle
from oracle import Kernel, EXP, M32, M52, SE
from paper_2606_11402_amd import KernelParams
from paper_2606_11402_amd import study

pytestmark = pytest.mark.gpu


def dense_kl(x, k, n0, kern):
    og = oracle.build_graph(x, k, n0)
    of = oracle.factor(og, kern)
    mat, d = oracle.vecchia.sparse_factor_matrices(og, of)
    f = np.linalg.solve(mat.toarray(), np.diag(d))
    kt = f @ f.T
    kd = oracle.dense_covariance(og.xs, kern)
    n = len(x)
    return 0.5 * (np.trace(np.linalg.solve(kt, kd)) - n + np.linalg.slogdet(kt)[1] - np.linalg.slogdet(kd)[1])


@pytest.mark.parametrize("kind,k", [(EXP, 4), (M32, 16), (M52, 8), (SE, 32)])
def test_kl_from_gpu_factor_matches_oracle(kind, k):
    x = np.random.default_rng(20 + k).standard_normal((400, 3))
    kern = Kernel(kind, 1.0, 1.0, 1e-6)
    kl, _, det = study.kl_divergence(x, k, 50, KernelParams(kind, 1.0, 1.0, 1e-6))
    ref = dense_kl(x, k, 50, kern)
    print("KL", kind, k, kl, ref, flush=True)
    assert kl > 0 and abs(kl - ref) <= 1e-6 * ref + 1e-9


@pytest.mark.parametrize("n0", [1, 20])
def test_kl_is_zero_in_the_exact_limit(n0):
    """N = 65, k = 64: every point conditions on all its predecessors."""
    n = 65
    x = np.random.default_rng(3).standard_normal((n, 3))
    kl, _, _ = study.kl_divergence(x, n - 1, n0, KernelParams(M32, 1.0, 1.0, 1e-6))
    assert abs(kl) <= 1e-8, kl


def test_kl_is_non_increasing_in_k():
    x = np.random.default_rng(4).standard_normal((1500, 3))
    kern = KernelParams(M32, 1.0, 1.0, 1e-8)
    exact = study.exact_cholesky(x, kern)
    vals = [study.kl_divergence(x, k, 50, kern, exact=exact)[0] for k in (2, 4, 8, 16, 32, 64)]
    print("KL vs k", vals, flush=True)
    assert all(v > 0 for v in vals)
    assert all(a >= b * (1 - 1e-6) for a, b in zip(vals, vals[1:])), vals
