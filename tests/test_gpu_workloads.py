"""Parity at the benchmark's full size (2048 x 1536, rank 1024, FP32) and the guarded stop rule."""
import numpy as np
import pytest

import qsynth
import fp32_chain as F32
from conftest import rel_fro, to_dev, to_np
from oracle import quat as Q
from oracle import methods as M

pytestmark = pytest.mark.gpu


#: Parity bound of an FP32 GPU result against the FP64 oracle, as a multiple of the error of the host evaluation
#: in which every product and stored intermediate is rounded to FP32 (tests/fp32_chain.py).  Both evaluations
#: make one rounding per stored value and accumulate dot products in FP32, in different orders; their errors
#: are sums of many independent rounding contributions pushed through the same chain, so they have the same
#: size in expectation.  The factor allows for the spread between two such evaluations.
FP32_SPREAD = 4.0


@pytest.fixture(scope="module")
def c2():
    inst = qsynth.c2_instance()
    inst["truth"] = Q.pinv_from_factors(inst["U"], inst["s"], inst["V"])  # the rank-1024 pseudoinverse
    return inst


def _oracle_and_fp32(A, X0, method, order, count):
    """X_count by the FP64 oracle and by the FP32 host evaluation, from the same X_0 (left residual side)."""
    Xo = X0
    for _ in range(count):
        Xo = M.step(A, Xo, method, order, "left")
    return Xo, F32.iterate(A, X0, method, count, order)


def test_full_size_one_step_fp32(qctx, c2):
    """One QHPI19 update at the timed launch configuration from an iterate both sides share, within
    FP32_SPREAD times the FP32 host evaluation's error."""
    import paper_2605_01464_amd as q

    A = c2["A"]
    X = M.x0(A, 1.0)
    for _ in range(4):  # a mid-convergence iterate, computed by the oracle
        X = M.step(A, X, "qhpi19", 19, "left")
    X = qsynth.round_f32(X)
    ref, x32 = _oracle_and_fp32(A, X, "qhpi19", 19, 1)
    Xd, _ = q.step(qctx, to_dev(A, "f32"), to_dev(X, "f32"), "qhpi19", side="left")
    e_gpu, e32 = rel_fro(to_np(Xd), ref), rel_fro(x32, ref)
    print(f"one update: GPU {e_gpu:.3e}, FP32 host evaluation {e32:.3e}")
    assert e_gpu <= FP32_SPREAD * e32, (e_gpu, e32)


@pytest.mark.parametrize("method,order", [("qhpi19", 19), ("ns", 2), ("qsai", 10), ("qrapid", 5)])
def test_full_size_returned_iterate(qctx, c2, method, order):
    """The benchmark's solve (power-iteration alpha, guarded stop at tol 1e-6, FP32) for every method: the
    returned X_j against the oracle's X_j from the same alpha on the identical FP32 input, within FP32_SPREAD
    times the FP32 host evaluation's error at the same j.  That error is large (about 1e-2 at the returned
    iterate): rounding seeds the ~1e-8 singular directions that rounding A to FP32 created, and every update
    multiplies them by its order there (19, 2, 10, 51.25)."""
    import sys

    import paper_2605_01464_amd as q

    A = c2["A"]
    X, info = q.solve(qctx, to_dev(A, "f32"), method, order, scaling="power", tol=1e-6, stop="guarded",
                      precision="f32", max_iter=200)
    assert info["status"] == q.OK and info["reason"] in ("rise", "tol"), info
    j = info["returned"]
    assert 1 <= j <= info["iters"]
    print(f"{method}: {info['iters']} updates, returned X_{j}; oracle and FP32 evaluation", file=sys.stderr, flush=True)
    ref, x32 = _oracle_and_fp32(A, M.x0(A, info["alpha_used"]), method, order, j)
    e_gpu, e32 = rel_fro(to_np(X), ref), rel_fro(x32, ref)
    print(f"{method} X_{j}: GPU {e_gpu:.3e}, FP32 host evaluation {e32:.3e}, GPU vs rank-1024 pinv "
          f"{rel_fro(to_np(X), c2['truth']):.3e}")
    assert e_gpu <= FP32_SPREAD * e32, (e_gpu, e32)


def test_full_size_penrose_finish(qctx, c2):
    """FP32 QHPI19, then FP64 Newton-Schulz updates with the projection X <- (X A)^H X (A X)^H before the last
    (option penrose_finish = 2): within the workload's 1e-4 of the oracle's result for the same schedule (X_{j*}
    of the FP32 phase's exit, the same FP64 updates and projection) and of the rank-1024 pseudoinverse
    V diag(1/s) U^H."""
    import torch

    import paper_2605_01464_amd as q

    A = c2["A"]
    try:
        qctx.set("penrose_finish", 2)
        X, info = q.solve(qctx, to_dev(A, "f32"), "qhpi19", scaling="power", tol=1e-6, stop="guarded",
                          precision="f32_f64finish", out_dtype=torch.float64)
    finally:
        qctx.set("penrose_finish", 0)
    assert info["status"] == q.OK and info["iters_f64"] >= 1, info
    j_star = info["returned"] - info["iters_f64"]
    assert 1 <= j_star <= info["iters_f32"], info
    Xo = M.x0(A, info["alpha_used"])
    for _ in range(j_star):
        Xo = M.step(A, Xo, "qhpi19", 19, "left")
    for k in range(info["iters_f64"]):
        if k == info["iters_f64"] - 1:
            Xo = M.penrose_projection(A, Xo)
        Xo = M.step(A, Xo, "ns", 2, "left")
    Xg = to_np(X)
    e_or, e_tr = rel_fro(Xg, Xo), rel_fro(Xg, c2["truth"])
    print(f"penrose finish: X_{j_star} + {info['iters_f64']} NS: vs oracle {e_or:.3e}, vs rank-1024 pinv {e_tr:.3e}")
    assert e_or <= 1e-4 and e_tr <= 1e-4, (e_or, e_tr, info)


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
