"""The paper's own timing workloads (Tables 1-2, Example 3) on seeded Gaussian stand-ins, FP64, with the
paper's stopping test ||X_{j+1} - X_j||_F < 1e-10: update counts against the oracle's exact-arithmetic
spectral model, and the Penrose residual of the result."""
import numpy as np
import pytest

import qsynth
from conftest import to_dev
from oracle import quat as Q
from oracle import methods as M

pytestmark = pytest.mark.gpu

# (m, n, alpha rule): Example 3 uses 1/sigma_1^2, Tables 1-2 fit 1/||A||_F^2 (the alpha is given to both
# sides, so the GPU and the model start from the same X_0)
WORKLOADS = [(800, 800, "sigma"), (1000, 500, "frob"), (500, 1000, "frob"), (300, 300, "frob")]
METHODS = [("qhpi19", None), ("qsai", None), ("qrapid", 5), ("ns", None)]


@pytest.mark.parametrize("m,n,rule", WORKLOADS)
def test_paper_workload_update_counts_equal_spectral_model(qctx, m, n, rule):
    import paper_2605_01464_amd as q

    A = qsynth.gaussian(9100 + m + n, m, n)
    s = Q.singular_values(A)
    alpha = 1.0 / s[0] ** 2 if rule == "sigma" else M.alpha_frobenius(A)
    Ad = to_dev(A, "f64")
    nA = Q.fro(A)
    for method, order in METHODS:
        J = M.spectral_dx_iterations(s, alpha, method, order, 1e-10)
        assert J <= 500
        X, info = q.solve(qctx, Ad, method, order, scaling="given", alpha=alpha, tol=1e-10, max_iter=500,
                          stop="dx_abs", precision="f64")
        assert info["status"] == q.OK and info["iters"] == J, (m, n, method, info["iters"], J)
        Ea, Er = q.residuals(qctx, Ad, X)
        assert Er[0] <= 1e-12 * max(1.0, s[0] / s[-1]), (m, n, method, Er, nA)
