"""The condition estimate used to grade the ill-conditioned (hard) variant is
pinned to the exact 1-norm condition number of the assembled operator of
eq. (1.4) at sizes where it can be formed."""
import numpy as np
import pytest

import tt_inputs as ti
from condest import inverse_norm1_estimate, laplace_norm1
from kron import laplace_dense


@pytest.mark.parametrize("shape,hard", [((5, 4, 6), None), ((6, 6, 6), 0.05), ((4, 5, 3, 4), 0.05),
                                        ((7, 8), 0.01)])
def test_condest_vs_dense(shape, hard):
    p = ti.laplace_tri(shape, seed=3, bumps="random", hard_sum=hard)
    L = laplace_dense(p["T"])
    assert laplace_norm1(p["T"]) == pytest.approx(np.linalg.norm(L, 1), rel=1e-13)
    exact = np.linalg.norm(np.linalg.inv(L), 1)
    est = inverse_norm1_estimate(p["T"], shape)
    # a lower bound by construction (norms of actual solves), usually exact
    assert exact / 3.0 <= est <= exact * (1 + 1e-10)
