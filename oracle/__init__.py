"""Plain, slow, FP64 CPU oracle for the Vecchia hot path of GraphGP.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product (``paper_2606_11402_amd``) never imports it, and this
package imports nothing from the product: the two share no code.  Inputs (the
points, the white noise) come from the seeded generators in ``workloads.py``,
which hold none of the method's arithmetic.

Every function follows a stated passage of the paper (GraphGP: Scalable
Gaussian Processes with Vecchia's Approximation):

* ``tree``       -- Sec. 2.2, "Tree ordering" and "Bit-reversed ordering".
* ``graph``      -- Sec. 2.1 (k nearest preceding neighbours) and Sec. 2.2,
                    "Batch construction" (depths and parallel batches).
* ``covariance`` -- the stationary kernels kappa(r) of Sec. 2.1 (forms named by
                    the benchmark workloads) and their parameter derivatives.
* ``vecchia``    -- Eq. (1)-(2), the dense initial batch and Alg. 1 (forward),
                    plus the inverse application and log-determinant listed as
                    building blocks in the abstract.
* ``adjoint``    -- kernel-parameter, white-noise and coordinate derivatives
                    (Sec. 2.3), written as closed forms of the conditional
                    formulas.
* ``tangent``    -- the forward-mode counterparts (Sec. 2.3: forward and
                    backward derivatives), same closed forms differentiated
                    in a direction.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, library routines or brute force (see the module
headers).  The paper prints no worked numerical example; the figure data
(batch sizes, KL divergences, timings) are absent, so those quantities are
"parity unpinned".
"""
from .covariance import (Kernel, EXP, M32, SE, M52, MATERN, kappa, dkappa_dsigma, dkappa_dell, dkappa_dr, cov_matrix,
                         cov_grad_x)
from .tree import tree_order, tree_level, left_child, right_child, parent
from .graph import Graph, build_graph, preceding_knn, depths, storage_order
from .vecchia import (Factor, dense_block, conditional, conditional_joint, factor,
                      forward, forward_sequential, forward_sparse_solve, inverse,
                      logdet, dense_covariance)
from .adjoint import forward_vjp, inverse_vjp, logdet_vjp, theta_grad, x_grad

from .tangent import factor_tangent, forward_jvp

__all__ = [
    "Kernel", "EXP", "M32", "SE", "M52", "MATERN", "kappa", "dkappa_dsigma", "dkappa_dell", "cov_matrix",
    "tree_order", "tree_level", "left_child", "right_child", "parent",
    "Graph", "build_graph", "preceding_knn", "depths", "storage_order",
    "Factor", "dense_block", "conditional", "conditional_joint", "factor", "forward",
    "forward_sequential", "forward_sparse_solve", "inverse", "logdet", "dense_covariance",
    "forward_vjp", "inverse_vjp", "logdet_vjp", "theta_grad", "factor_tangent", "forward_jvp",
]
