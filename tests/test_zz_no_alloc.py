"""The allocation-free solve entry point against qpinv_solve (same kernels and tiles: identical results)."""
import numpy as np
import pytest

import qsynth
from conftest import rel_fro, to_dev, to_np
from oracle import methods as M

pytestmark = pytest.mark.gpu


def _compare(ctx, A, precision, method, tol, stop, order=None):
    import torch

    import paper_2605_01464_amd as q

    Ad = to_dev(A, "f64" if precision == "f64" else "f32")
    X_ref, info_ref = q.solve(ctx, Ad, method, order, scaling="power", tol=tol, stop=stop, precision=precision)
    X = torch.full_like(X_ref, float("nan"))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    info = q.solve_noalloc(ctx, Ad, X, method, order, scaling="power", tol=tol, stop=stop, precision=precision)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert info["status"] == info_ref["status"] == q.OK, (info, info_ref)
    for k in ("iters", "returned", "stop_reason", "side", "alpha_used", "iters_f32", "iters_f64"):
        assert info[k] == info_ref[k], (k, info[k], info_ref[k])
    assert torch.equal(X, X_ref)
    return X, info


def test_noalloc_matches_solve_two_calls(qctx):
    """Two calls in a row, the second on a smaller matrix (the scratch holds the first call's buffers): each
    result equals qpinv_solve's bit for bit, and the FP64 one follows the oracle run from the same alpha."""
    import paper_2605_01464_amd as q

    qctx.set("autotune", 0)
    A1 = qsynth.c1_instance(4)  # 64 x 48, planes N(0,1)
    X1, info1 = _compare(qctx, A1, "f64", "qhpi19", 1e-12, "e1_rel")
    ro = M.solve(A1, "qhpi19", alpha=info1["alpha_used"], tol=1e-12, stop="e1_rel", side="left")
    assert info1["iters"] == ro.iters
    assert rel_fro(to_np(X1), ro.X) <= 1e-12
    A2 = qsynth.round_f32(np.random.default_rng(31).standard_normal((4, 33, 21)))
    X2, info2 = _compare(qctx, A2, "f32", "qsai", 1e-6, "guarded")
    ref2 = M.solve(A2, "qsai", alpha=info2["alpha_used"], tol=1e-12, stop="e1_rel", side="left").X
    assert rel_fro(to_np(X2), ref2) <= 5e-5
    # the FP32 iterations with the FP64 finish, wide shape (right-side residual), after the smaller call
    A3 = qsynth.round_f32(np.random.default_rng(32).standard_normal((4, 40, 72)))
    _compare(qctx, A3, "f32_f64finish", "qhpi19", 1e-6, "guarded")


def test_noalloc_qrapid_one_launch(qctx):
    """QRAPID's one-launch solves without allocation: QRAPID(5) on the 64 x 48 FP64 input (16 phases per update,
    left side), then QRAPID(8) on a smaller wide matrix (24 phases, right side) and QRAPID(0) on the first
    again, each equal to qpinv_solve's result bit for bit; the first follows the oracle from the same alpha."""
    qctx.set("autotune", 0)
    A1 = qsynth.c1_instance(6)
    X1, info1 = _compare(qctx, A1, "f64", "qrapid", 1e-12, "e1_rel", order=5)
    ro = M.solve(A1, "qrapid", 5, alpha=info1["alpha_used"], tol=1e-12, stop="e1_rel", side="left")
    assert info1["iters"] == ro.iters
    assert rel_fro(to_np(X1), ro.X) <= 1e-12
    A2 = np.random.default_rng(34).standard_normal((4, 29, 37))
    _compare(qctx, A2, "f64", "qrapid", 1e-12, "dx_rel", order=8)
    _compare(qctx, A1, "f64", "qrapid", 1e-12, "dx_rel", order=0)


def test_noalloc_ladder_uses_native_fp32_products(qctx):
    """The BF16 -> FP32 -> FP64 ladder without allocation: its FP32-storage products stay native FP32 (the split
    BF16 products would need the stage buffer to grow), so it equals qpinv_solve with option mixed_split = 0 bit
    for bit, on a fresh context as well as after the other calls."""
    import paper_2605_01464_amd as q

    qctx.set("autotune", 0)
    A = qsynth.round_f32(np.random.default_rng(33).standard_normal((4, 150, 130)))
    try:
        qctx.set("mixed_split", 0)
        _compare(qctx, A, "mixed", "qhpi19", 1e-6, "guarded")
    finally:
        qctx.set("mixed_split", 1)
    fresh = q.Context(0)
    try:
        fresh.set("autotune", 0)
        fresh.set("mixed_split", 0)
        _compare(fresh, A, "mixed", "qhpi19", 1e-6, "guarded")
    finally:
        fresh.close()


def test_noalloc_rejects_oversize_before_launch(qctx):
    """A shape whose workspace bound exceeds the scratch is refused with EINVAL; X is left untouched."""
    import torch

    import paper_2605_01464_amd as q

    A = torch.zeros((4, 300, 300), dtype=torch.float64, device="cuda")
    X = torch.full((4, 300, 300), 7.0, dtype=torch.float64, device="cuda")
    info = q.solve_noalloc(qctx, A, X, "qhpi19", precision="f64", check=False)
    assert info["status"] == q.EINVAL
    assert "no-allocation scratch" in q.qpinv_last_error()
    torch.cuda.synchronize()
    assert float((X - 7.0).abs().max()) == 0.0
