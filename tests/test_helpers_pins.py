"""Pins of the test helpers that assess GPU results (run on the CPU): the
backward error of coefficient rows is at roundoff level for the oracle's own
coefficients, even where K_cc is ill-conditioned, and large for a
coefficient row with one wrong entry."""
import numpy as np

import oracle
import workloads
from oracle import Kernel, M32
from gpu_helpers import b_backward_error


def test_b_backward_error_of_oracle_coefficients_and_of_a_wrong_entry():
    w = workloads.WORKLOADS[2]
    x = w.points(3000)
    og = oracle.build_graph(x, 16, 128)
    kern = Kernel(M32, 1.0, 0.05)
    fac = oracle.factor(og, kern)
    assert b_backward_error(og, kern, fac.b) < 1e-13
    bad = fac.b.copy()
    bad[100, 3] += 1e-6 * np.abs(bad[100]).max()
    assert b_backward_error(og, kern, bad) > 1e-9
    sign = fac.b.copy()
    sign[7, 0] = -sign[7, 0]
    assert b_backward_error(og, kern, sign) > 1e-3
