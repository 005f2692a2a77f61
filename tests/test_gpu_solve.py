"""One iteration and full solves on the GPU vs the FP64 oracle (same inputs, same alpha, same side)."""
import numpy as np
import pytest

import qsynth
from conftest import rel_fro, to_dev, to_np
from oracle import quat as Q
from oracle import methods as M

pytestmark = pytest.mark.gpu

CASES = [("ns", None), ("hpi", 5), ("qsai", None), ("qhpi19", None), ("qrapid", 0), ("qrapid", 2), ("qrapid", 5)]


def _order(method, order):
    return {"ns": 2, "qsai": 10, "qhpi19": 19, "qrapid": 5}.get(method) if order is None else order


@pytest.mark.parametrize("method,order", CASES)
@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("shape", [(70, 45), (45, 70), (64, 64)])
def test_one_step_fp64(qctx, method, order, side, shape):
    import paper_2605_01464_amd as q

    A = np.random.default_rng(11).standard_normal((4,) + shape)
    X0 = M.x0(A, 0.9 * M.alpha_sigma(A))
    X1 = M.step(A, X0, method, _order(method, order), side)
    Xd, dx = q.step(qctx, to_dev(A, "f64"), to_dev(X0, "f64"), method, _order(method, order), side=side)
    assert rel_fro(to_np(Xd), X1) <= 1e-12
    assert dx[0] == pytest.approx(Q.fro(X1 - X0) ** 2, rel=1e-9)
    assert dx[1] == pytest.approx(Q.fro(X1) ** 2, rel=1e-12)


@pytest.mark.parametrize("method,order", CASES)
@pytest.mark.parametrize("side", ["left", "right"])
def test_one_step_fp32(qctx, method, order, side):
    import paper_2605_01464_amd as q

    A = qsynth.round_f32(np.random.default_rng(12).standard_normal((4, 150, 97)))
    X0 = qsynth.round_f32(M.x0(A, 0.9 * M.alpha_sigma(A)))
    X1 = M.step(A, X0, method, _order(method, order), side)
    Xd, _ = q.step(qctx, to_dev(A, "f32"), to_dev(X0, "f32"), method, _order(method, order), side=side)
    # up to 8 + 2N chained FP32 products of well-scaled operands
    assert rel_fro(to_np(Xd), X1) <= 2e-5


@pytest.mark.parametrize("side", ["left", "right"])
def test_residual_law_on_gpu_iterate(qctx, side):
    """I - A X_{j+1} = (I - A X_j)^19 holds for the GPU's QHPI19 iterate from a generic X_j (FP64)."""
    import paper_2605_01464_amd as q

    A = np.random.default_rng(13).standard_normal((4, 40, 30))
    X = Q.pinv_svd(A) + 0.01 / Q.fro(A) * np.random.default_rng(14).standard_normal((4, 30, 40))
    Xd, _ = q.step(qctx, to_dev(A, "f64"), to_dev(X, "f64"), "qhpi19", side=side)
    I = Q.qeye(40)
    R = I - Q.qmul(A, X)
    R19 = I.copy()
    for _ in range(19):
        R19 = Q.qmul(R19, R)
    Rn = I - Q.qmul(A, to_np(Xd))
    assert Q.fro(Rn - R19) <= 1e-11


def test_residuals_match_oracle(qctx):
    import paper_2605_01464_amd as q

    A = np.random.default_rng(15).standard_normal((4, 50, 35))
    X = Q.pinv_svd(A) + 1e-3 * np.random.default_rng(16).standard_normal((4, 35, 50))
    Ea, Er = q.residuals(qctx, to_dev(A, "f64"), to_dev(X, "f64"))
    o = M.residuals(A, X)
    np.testing.assert_allclose(Ea, o["E"], rtol=1e-9)
    np.testing.assert_allclose(Er, o["E_rel"], rtol=1e-9)
    # FP32 inputs are widened exactly
    Ea32, _ = q.residuals(qctx, to_dev(A, "f32"), to_dev(X, "f32"))
    o32 = M.residuals(qsynth.round_f32(A), qsynth.round_f32(X))
    np.testing.assert_allclose(Ea32, o32["E"], rtol=1e-9)


# ------------------------------------------------------------------ small workload: 64 x 48, FP64
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("method,order", [("ns", None), ("qsai", None), ("qhpi19", None), ("qrapid", 5)])
def test_small_workload_fp64(qctx, seed, method, order):
    import paper_2605_01464_amd as q

    A = qsynth.c1_instance(seed)
    alpha = M.alpha_sigma(A)
    ro = M.solve(A, method, _order(method, order), alpha=alpha, tol=1e-12, stop="e1_rel", side="left")
    X, info = q.solve(qctx, to_dev(A, "f64"), method, _order(method, order), scaling="given", alpha=alpha,
                      tol=1e-12, stop="e1_rel", precision="f64")
    assert info["status"] == q.OK and info["reason"] == "tol"
    assert info["side"] == q.SIDE["left"]
    assert info["iters"] == ro.iters
    Xg = to_np(X)
    assert rel_fro(Xg, ro.X) <= 1e-12
    assert rel_fro(Xg, Q.pinv_full_column_rank(A)) <= 1e-10
    Ea, Er = q.residuals(qctx, to_dev(A, "f64"), X)
    assert Er[0] <= 1e-12 and max(Er) <= 1e-12


def test_small_workload_power_alpha(qctx):
    import paper_2605_01464_amd as q

    A = qsynth.c1_instance(3)
    f = M.features(A, 8)
    ro = M.solve(A, "qhpi19", alpha=1.0 / f["sigma1_sq"], tol=1e-12, stop="e1_rel", side="left")
    X, info = q.solve(qctx, to_dev(A, "f64"), "qhpi19", scaling="power", tol=1e-12, stop="e1_rel", precision="f64")
    assert info["alpha_used"] == pytest.approx(1.0 / f["sigma1_sq"], rel=1e-12)
    assert info["iters"] == ro.iters
    assert rel_fro(to_np(X), ro.X) <= 1e-12


@pytest.mark.parametrize("dtype,shape", [("f64", (64, 48)), ("f32", (150, 97)), ("f64", (3, 3))])
def test_frobenius_scaling_matches_oracle(qctx, example1, dtype, shape):
    """Section 4's alpha = 1/||A||_F^2 (scaling FROB): the GPU's alpha_used equals the oracle's on the values the
    GPU holds (FP32 inputs widened exactly), and the solve from it follows the oracle run from the same alpha."""
    import paper_2605_01464_amd as q

    if shape == (3, 3):
        A = example1[0]
    else:
        A = np.random.default_rng(18).standard_normal((4,) + shape)
    if dtype == "f32":
        A = qsynth.round_f32(A)
    a_ref = M.alpha_frobenius(A)
    if shape == (3, 3):
        assert a_ref == pytest.approx(1.0 / 532.0, rel=1e-15)
    X, info = q.solve(qctx, to_dev(A, dtype), "qhpi19", scaling="frob", tol=1e-12 if dtype == "f64" else 1e-6,
                      stop="e1_rel" if dtype == "f64" else "guarded", precision=dtype, max_iter=100)
    assert info["alpha_used"] == pytest.approx(a_ref, rel=1e-13)
    if dtype == "f64":
        ro = M.solve(A, "qhpi19", alpha=a_ref, tol=1e-12, stop="e1_rel", side="left" if shape[0] > shape[1] else "right")
        assert info["iters"] == ro.iters
        assert rel_fro(to_np(X), ro.X) <= 1e-12


def test_worked_example_on_gpu(qctx, example1):
    """Section 4, Example 1 through the GPU path: printed pseudoinverse and iteration counts."""
    import paper_2605_01464_amd as q

    A, P, _, iters = example1
    alpha = M.alpha_sigma(A)
    qctx.set("side", q.SIDE["right"])
    try:
        for method, order in [("qsai", 10), ("qhpi19", 19), ("qrapid", 2)]:
            X, info = q.solve(qctx, to_dev(A, "f64"), method, order, scaling="given", alpha=alpha, tol=1e-10,
                              stop="dx_abs", precision="f64")
            assert info["iters"] == iters[method]
            assert np.max(np.abs(to_np(X) - P)) <= 5e-5 + 1e-9
    finally:
        qctx.set("side", q.SIDE["auto"])


# ------------------------------------------------------------------ error paths
def test_error_paths(qctx):
    import torch
    import paper_2605_01464_amd as q

    A = np.random.default_rng(17).standard_normal((4, 30, 20))
    Ad = to_dev(A, "f64")
    s1 = Q.singular_values(A)[0]
    # alpha outside (0, 2/sigma_1^2): Theorem 1 -> divergence
    _, info = q.solve(qctx, Ad, "qhpi19", scaling="given", alpha=2.5 / s1 ** 2, tol=1e-12, stop="dx_rel",
                      precision="f64", check=False)
    assert info["status"] == q.EDIVERGED
    # max_iter exhausted
    _, info = q.solve(qctx, Ad, "ns", scaling="given", alpha=1.0 / s1 ** 2, tol=0.0, max_iter=2, stop="dx_rel",
                      precision="f64", check=False)
    assert info["status"] == q.ENOTCONVERGED and info["iters"] == 2
    # non-finite input
    Abad = A.copy()
    Abad[1, 4, 5] = np.inf
    _, info = q.solve(qctx, to_dev(Abad, "f64"), "qhpi19", precision="f64", check=False)
    assert info["status"] == q.ENONFINITE
    # bad order / shape
    X = torch.empty((4, 20, 30), dtype=torch.float64, device="cuda")
    st, _ = q.qpinv_solve(qctx.handle, q.METHOD["qsai"], 7, Ad, 0, 0.0, 1e-6, 10, 3, 0, X)
    assert st == q.EINVAL
    Xbad = torch.empty((4, 30, 20), dtype=torch.float64, device="cuda")
    st, _ = q.qpinv_solve(qctx.handle, q.METHOD["qhpi19"], 19, Ad, 0, 0.0, 1e-6, 10, 3, 0, Xbad)
    assert st == q.EINVAL
    # zero matrix: pseudoinverse is zero
    Z = torch.zeros((4, 6, 4), dtype=torch.float64, device="cuda")
    Xz, info = q.solve(qctx, Z, "qhpi19", precision="f64")
    assert float(Xz.abs().max()) == 0.0


@pytest.mark.parametrize("method", ["qhpi19", "qsai", "ns", "qrapid"])
def test_degenerate_shapes(qctx, method):
    """1 x 1, column and row vectors (closed form a^H / ||a||^2, Section 2), and empty matrices."""
    import torch

    import paper_2605_01464_amd as q

    rng = np.random.default_rng(19)
    for shape in ((1, 1), (9, 1), (1, 7)):
        A = rng.standard_normal((4,) + shape)
        X, info = q.solve(qctx, to_dev(A, "f64"), method, tol=1e-13, max_iter=200, stop="e1_rel", precision="f64")
        ref = Q.qH(A) / np.sum(A * A)
        assert info["status"] == q.OK, (shape, info)
        assert Q.fro(to_np(X) - ref) <= 1e-12 * Q.fro(ref), shape
    for shape in ((0, 5), (5, 0)):
        A = torch.zeros((4,) + shape, dtype=torch.float64, device="cuda")
        X, info = q.solve(qctx, A, method, precision="f64")
        assert tuple(X.shape) == (4, shape[1], shape[0]) and info["status"] == q.OK


# ------------------------------------------------------------------ Penrose projection of the result
@pytest.fixture(scope="module")
def rank_def():
    """150 x 110 of rank 60 (s geometric 1 .. 1e-3), rounded to FP32: numerically rank deficient."""
    inst = qsynth.small_spectral_instance(120, 150, 110, qsynth.geometric(60, 1.0, 1e-3))
    inst["A"] = qsynth.round_f32(inst["A"])
    return inst


@pytest.mark.parametrize("mode", [1, 2])
def test_penrose_finish_fp64(qctx, rank_def, mode):
    """FP64 solve with the guarded stop, then X A X (mode 1) or the projection (X A)^H X (A X)^H and one
    Newton-Schulz update (mode 2): the oracle's returned iterate with the same steps."""
    import paper_2605_01464_amd as q

    A = rank_def["A"]
    alpha = M.alpha_sigma(A)
    ro = M.solve(A, "qhpi19", alpha=alpha, tol=1e-15, stop="guarded", side="left", max_iter=80)
    try:
        qctx.set("penrose_finish", mode)
        X, info = q.solve(qctx, to_dev(A, "f64"), "qhpi19", scaling="given", alpha=alpha, tol=1e-15, stop="guarded",
                          precision="f64", max_iter=80)
    finally:
        qctx.set("penrose_finish", 0)
    if mode == 1:
        ref = Q.qmul(Q.qmul(ro.X, A), ro.X)
        assert info["iters"] == ro.iters and info["returned"] == ro.returned
    else:
        ref = M.step(A, M.penrose_projection(A, ro.X), "ns", 2, "left")
        assert info["iters"] == ro.iters + 1 and info["returned"] == ro.returned + 1
    assert rel_fro(to_np(X), ref) <= 1e-8
    truth = Q.pinv_from_factors(rank_def["U"], rank_def["s"], rank_def["V"])
    print(f"mode {mode}: vs oracle {rel_fro(to_np(X), ref):.2e}, vs rank-60 pinv {rel_fro(to_np(X), truth):.2e}")


def test_penrose_finish_in_fp64_finish(qctx, rank_def):
    """FP32 QHPI19 with the FP64 finish and the projection before its last update: the oracle's schedule from
    the FP32 phase's exit iterate, and closer to the rank-60 pseudoinverse than the finish without it."""
    import torch

    import paper_2605_01464_amd as q

    A = rank_def["A"]
    truth = Q.pinv_from_factors(rank_def["U"], rank_def["s"], rank_def["V"])
    out = {}
    for mode in (0, 2):
        try:
            qctx.set("penrose_finish", mode)
            X, info = q.solve(qctx, to_dev(A, "f32"), "qhpi19", scaling="power", tol=1e-6, stop="guarded",
                              precision="f32_f64finish", out_dtype=torch.float64)
        finally:
            qctx.set("penrose_finish", 0)
        out[mode] = (to_np(X), info)
    X2, info = out[2]
    assert info["status"] == q.OK and info["iters_f64"] == 2, info
    j_star = info["returned"] - info["iters_f64"]
    Xo = M.x0(A, info["alpha_used"])
    for _ in range(j_star):
        Xo = M.step(A, Xo, "qhpi19", 19, "left")
    Xo = M.step(A, Xo, "ns", 2, "left")
    Xo = M.step(A, M.penrose_projection(A, Xo), "ns", 2, "left")
    assert rel_fro(X2, Xo) <= 1e-4
    assert rel_fro(X2, truth) < rel_fro(out[0][0], truth)


def test_penrose_projection_needs_fp64_updates(qctx, rank_def):
    import paper_2605_01464_amd as q

    try:
        qctx.set("penrose_finish", 2)
        _, info = q.solve(qctx, to_dev(rank_def["A"], "f32"), "qhpi19", precision="f32", check=False)
    finally:
        qctx.set("penrose_finish", 0)
    assert info["status"] == q.EINVAL


# ------------------------------------------------------------------ one-launch path for small matrices
SMALL_SHAPES = [(64, 48), (48, 64), (37, 29), (29, 37), (128, 128), (128, 97), (1, 1), (9, 1), (1, 7)]


@pytest.mark.parametrize("shape", SMALL_SHAPES)
@pytest.mark.parametrize("method,order", [("ns", 2), ("qsai", 10), ("qhpi19", 19), ("qrapid", 5)])
@pytest.mark.parametrize("stop,scaling", [("e1_rel", "power"), ("dx_rel", "frob"), ("dx_abs", "given")])
def test_small_path_matches_oracle_and_regular_path(qctx, shape, method, order, stop, scaling):
    """FP64 solves of at most 128 per side run as one launch (small_path = 1, the default): the same update
    count and returned iterate as the oracle from the same alpha (<= 1e-12) and as the product-by-product
    path (small_path = 0)."""
    _small_vs_regular(qctx, shape, method, order, stop, scaling)


@pytest.mark.parametrize("shape", [(64, 48), (29, 37), (128, 97), (1, 7)])
@pytest.mark.parametrize("order", [0, 1, 8, 9])
@pytest.mark.parametrize("stop,scaling", [("e1_rel", "power"), ("dx_rel", "frob")])
def test_small_path_qrapid_orders(qctx, shape, order, stop, scaling):
    """QRAPID(N) in one launch for N <= 8 (6 + 2N phases on the left side, 8 + 2N on the right, at most 24);
    N = 9 takes the product-by-product path.  Both match the oracle and each other."""
    _small_vs_regular(qctx, shape, "qrapid", order, stop, scaling)


def test_small_path_qrapid_runs_one_launch(qctx, capfd):
    """QRAPID(8) of a 48 x 64 matrix (24 phases, the table's limit) runs as one launch and QRAPID(9) does
    not: the one-launch path's trace line (option verbose) is printed for the first only."""
    import paper_2605_01464_amd as q

    Ad = to_dev(np.random.default_rng(45).standard_normal((4, 48, 64)), "f64")
    kw = dict(scaling="power", tol=1e-12, stop="dx_rel", precision="f64")
    qctx.set("verbose", 1)
    try:
        capfd.readouterr()
        _, info = q.solve(qctx, Ad, "qrapid", 8, **kw)
        err8 = capfd.readouterr().err
        _, info9 = q.solve(qctx, Ad, "qrapid", 9, **kw)
        err9 = capfd.readouterr().err
    finally:
        qctx.set("verbose", 0)
    assert info["status"] == q.OK and info9["status"] == q.OK
    assert "small solve" in err8 and "small solve" not in err9


@pytest.mark.parametrize("shape", [(64, 48), (29, 37), (128, 97)])
@pytest.mark.parametrize("method,order", [("ns", 2), ("qhpi19", 19), ("qrapid", 5)])
def test_small_path_gram_setup_matches_plain_setup(qctx, shape, method, order):
    """The Gram matrix formed during the set-up (option small_gram = 1, the default; A^H A on the left side,
    A A^H on the right) against the first side product formed from X_0 (0): the same update count, and
    iterates within 1e-12 of each other and of the oracle from the same alpha."""
    import paper_2605_01464_amd as q

    A = np.random.default_rng(46 + shape[0]).standard_normal((4,) + shape)
    kw = dict(scaling="power", tol=1e-12, stop="e1_rel", precision="f64", max_iter=100)
    Ad = to_dev(A, "f64")
    X1, i1 = q.solve(qctx, Ad, method, order, **kw)
    try:
        qctx.set("small_gram", 0)
        X0, i0 = q.solve(qctx, Ad, method, order, **kw)
    finally:
        qctx.set("small_gram", 1)
    assert i1["status"] == i0["status"] == q.OK
    assert i1["iters"] == i0["iters"] and i1["alpha_used"] == i0["alpha_used"]
    assert rel_fro(to_np(X1), to_np(X0)) <= 1e-12
    side = "left" if shape[0] > shape[1] else "right"
    ro = M.solve(A, method, order, alpha=i1["alpha_used"], tol=1e-12, stop="e1_rel", side=side, max_iter=100)
    assert i1["iters"] == ro.iters and rel_fro(to_np(X1), ro.X) <= 1e-12


def _small_vs_regular(qctx, shape, method, order, stop, scaling):
    import paper_2605_01464_amd as q

    A = np.random.default_rng(40 + shape[0] + 3 * shape[1]).standard_normal((4,) + shape)
    alpha = 0.9 * M.alpha_sigma(A) if scaling == "given" else 0.0
    tol = {"e1_rel": 1e-12, "dx_rel": 1e-12, "dx_abs": 1e-10 * Q.fro(Q.pinv_svd(A))}[stop]
    kw = dict(scaling=scaling, alpha=alpha, tol=tol, stop=stop, precision="f64", max_iter=100)
    Ad = to_dev(A, "f64")
    X, info = q.solve(qctx, Ad, method, order, **kw)
    try:
        qctx.set("small_path", 0)
        Xr, ir = q.solve(qctx, Ad, method, order, **kw)
    finally:
        qctx.set("small_path", 1)
    side = "left" if shape[0] > shape[1] else "right"
    ro = M.solve(A, method, order, alpha=info["alpha_used"], tol=tol, stop=stop, side=side, max_iter=100)
    assert info["status"] == q.OK and info["reason"] == "tol", info
    assert info["iters"] == ro.iters == ir["iters"], (info["iters"], ro.iters, ir["iters"])
    assert info["returned"] == ir["returned"] and info["side"] == ir["side"]
    assert info["alpha_used"] == pytest.approx(ir["alpha_used"], rel=1e-13)
    assert rel_fro(to_np(X), ro.X) <= 1e-12
    assert rel_fro(to_np(X), to_np(Xr)) <= 1e-12
    if stop == "e1_rel":
        assert info["e1_rel"] <= tol


@pytest.mark.parametrize("method,order", [("qhpi19", 19), ("ns", 2), ("qsai", 10), ("qrapid", 5)])
def test_small_path_fp32(qctx, method, order):
    """FP32 one-launch solves of a 100 x 70 matrix: the regular path's update count, and both within FP32
    rounding of the oracle's iterate."""
    import paper_2605_01464_amd as q

    A = qsynth.round_f32(np.random.default_rng(43).standard_normal((4, 100, 70)))
    kw = dict(scaling="power", tol=1e-6, stop="dx_rel", precision="f32", max_iter=100)
    X, info = q.solve(qctx, to_dev(A, "f32"), method, order, **kw)
    try:
        qctx.set("small_path", 0)
        Xr, ir = q.solve(qctx, to_dev(A, "f32"), method, order, **kw)
    finally:
        qctx.set("small_path", 1)
    ro = M.solve(A, method, order, alpha=info["alpha_used"], tol=1e-12, stop="e1_rel", side="left")
    assert info["status"] == q.OK and info["iters"] == ir["iters"], (info, ir)
    assert rel_fro(to_np(X), ro.X) <= 2e-5 and rel_fro(to_np(Xr), ro.X) <= 2e-5


def test_small_path_barrier_giveup_reports_timeout(qctx):
    """A grid-barrier wait of the one-launch path that gives up: forced from the host (the give-up flag
    raised before the launch), every workgroup leaves at its first barrier and no result record is written;
    the call reports ETIMEOUT, and the next solve on the same context (which clears the barrier words)
    matches the oracle."""
    import paper_2605_01464_amd as q

    A = qsynth.c1_instance(5)
    Ad = to_dev(A, "f64")
    kw = dict(scaling="power", tol=1e-12, stop="e1_rel", precision="f64")
    qctx.set("fault_small_giveup", 1)
    try:
        _, info = q.solve(qctx, Ad, "qhpi19", check=False, **kw)
    finally:
        qctx.set("fault_small_giveup", 0)
    assert info["status"] == q.ETIMEOUT
    X, info = q.solve(qctx, Ad, "qhpi19", **kw)
    assert info["status"] == q.OK and info["reason"] == "tol"
    ro = M.solve(A, "qhpi19", alpha=info["alpha_used"], tol=1e-12, stop="e1_rel", side="left")
    assert info["iters"] == ro.iters
    assert rel_fro(to_np(X), ro.X) <= 1e-12


def test_small_path_error_paths(qctx):
    """The one-launch path's statuses: divergence for alpha outside Theorem 1's interval, max_iter, a
    non-finite input, a zero matrix (pseudoinverse 0), an FP32 input solved in FP64 (converted first)."""
    import torch

    import paper_2605_01464_amd as q

    A = np.random.default_rng(44).standard_normal((4, 30, 20))
    Ad = to_dev(A, "f64")
    s1 = Q.singular_values(A)[0]
    _, info = q.solve(qctx, Ad, "qhpi19", scaling="given", alpha=2.5 / s1 ** 2, tol=1e-12, stop="dx_rel",
                      precision="f64", check=False)
    assert info["status"] == q.EDIVERGED and info["reason"] == "diverged"
    _, info = q.solve(qctx, Ad, "ns", scaling="given", alpha=1.0 / s1 ** 2, tol=0.0, max_iter=2, stop="e1_rel",
                      precision="f64", check=False)
    assert info["status"] == q.ENOTCONVERGED and info["iters"] == 2
    Abad = A.copy()
    Abad[2, 7, 3] = np.nan
    _, info = q.solve(qctx, to_dev(Abad, "f64"), "qhpi19", stop="e1_rel", precision="f64", check=False)
    assert info["status"] == q.ENONFINITE
    Z = torch.zeros((4, 6, 4), dtype=torch.float64, device="cuda")
    Xz, info = q.solve(qctx, Z, "qhpi19", stop="e1_rel", tol=1e-12, precision="f64")
    assert info["status"] == q.OK and float(Xz.abs().max()) == 0.0
    X64, info = q.solve(qctx, to_dev(A, "f32"), "qhpi19", stop="e1_rel", tol=1e-12, precision="f64",
                        out_dtype=torch.float64)
    ro = M.solve(qsynth.round_f32(A), "qhpi19", alpha=info["alpha_used"], tol=1e-12, stop="e1_rel", side="left")
    assert info["iters"] == ro.iters and rel_fro(to_np(X64), ro.X) <= 1e-12
