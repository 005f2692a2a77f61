"""Parity at the benchmark's full size (2048 x 1536, rank 1024, FP32) and the guarded stop rule."""
import numpy as np
import pytest

import qsynth
from conftest import rel_fro, to_dev, to_np
from oracle import quat as Q
from oracle import methods as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    return qsynth.c2_instance()


def test_full_size_one_step_fp32(qctx, c2):
    """One QHPI19 update at the timed launch configuration from an iterate both sides share."""
    import paper_2605_01464_amd as q

    A = c2["A"]
    X = M.x0(A, 1.0)
    for _ in range(4):  # a mid-convergence iterate, computed by the oracle
        X = M.step(A, X, "qhpi19", 19, "left")
    X = qsynth.round_f32(X)
    ref = M.step(A, X, "qhpi19", 19, "left")
    Xd, _ = q.step(qctx, to_dev(A, "f32"), to_dev(X, "f32"), "qhpi19", side="left")
    # seven chained FP32 products with K up to 2048 on an iterate with entries up to ~1e3: host sgemm
    # (blocked accumulation) lands at 4e-5 here; one accumulator per MFMA tile over the whole K range
    # accumulates longer rounding chains
    assert rel_fro(to_np(Xd), ref) <= 3e-4


@pytest.mark.parametrize("J,tol", [(3, 1e-4), (5, 1e-3), (6, 5e-3)])
def test_full_size_fixed_iterations_fp32(qctx, c2, J, tol):
    """X_J of the FP32 GPU solve vs X_J of the FP64 oracle on the same FP32 input, same alpha.
    The FP32 tolerance grows with J: rounding seeds the ~1e-8 singular directions that rounding A
    to FP32 created, and QHPI19 multiplies them by ~19 per update."""
    import paper_2605_01464_amd as q

    A = c2["A"]
    Xo = M.x0(A, 1.0)
    for _ in range(J):
        Xo = M.step(A, Xo, "qhpi19", 19, "left")
    X, info = q.solve(qctx, to_dev(A, "f32"), "qhpi19", scaling="given", alpha=1.0, tol=0.0, max_iter=J,
                      stop="dx_rel", precision="f32", check=False)
    assert info["status"] == q.ENOTCONVERGED and info["iters"] == J
    assert rel_fro(to_np(X), Xo) <= tol


def test_full_size_solve_reaches_fp32_floor(qctx, c2):
    """The benchmark's solve: guarded stop returns an iterate within the FP32 floor of this problem."""
    import paper_2605_01464_amd as q

    X, info = q.solve(qctx, to_dev(c2["A"], "f32"), "qhpi19", scaling="power", tol=1e-6, stop="guarded",
                      precision="f32")
    assert info["reason"] in ("rise", "tol")
    Xt = Q.pinv_from_factors(c2["U"], c2["s"], c2["V"])
    assert rel_fro(to_np(X), Xt) <= 5e-2


@pytest.mark.parametrize("method,order", [("qhpi19", 19), ("qsai", 10), ("ns", 2)])
def test_guarded_stop_fp64_matches_oracle(qctx, method, order):
    """FP64 on a rounded rank-deficient matrix: the relative change falls, then rises as the rounding-made
    singular values start to be inverted.  GPU and oracle stop at the same update and return the same
    iterate."""
    import paper_2605_01464_amd as q

    inst = qsynth.small_spectral_instance(7, 256, 192, qsynth.geometric(128, 1.0, 1e-4))
    A = qsynth.round_f32(inst["A"])
    alpha = M.alpha_sigma(A)
    ro = M.solve(A, method, order, alpha=alpha, tol=1e-15, stop="guarded", side="left", max_iter=80)
    X, info = q.solve(qctx, to_dev(A, "f64"), method, order, scaling="given", alpha=alpha, tol=1e-15,
                      stop="guarded", precision="f64", max_iter=80)
    assert ro.reason == "rise"
    assert info["reason"] == "rise"
    assert info["iters"] == ro.iters and info["returned"] == ro.returned
    assert rel_fro(to_np(X), ro.X) <= 1e-8
