"""Batched solves in one persistent launch vs the FP64 oracle, matrix by matrix."""
import numpy as np
import pytest

import qsynth
from conftest import rel_fro, to_dev, to_np
from oracle import quat as Q
from oracle import methods as M

pytestmark = pytest.mark.gpu

# kernel forms: the queue kernel (one workgroup per matrix), the phase-synchronous kernel (all
# workgroups per product, a grid barrier after each) and its dataflow form (per-matrix completion counters,
# one grid barrier per update), with the same 32 x 32 tile routine
FORMS = {"queue": 0, "sync": 3, "sync_bk32": 5, "flow": 6, "flow_bk16": 7}
PREFIX = {"queue": "batched_f32", "sync": "batched_sync", "flow": "batched_flow"}


@pytest.fixture(autouse=True, params=sorted(FORMS))
def batched_form(request, qctx):
    import paper_2605_01464_amd as q

    cfg = FORMS[request.param]
    assert q.qpinv_batched_config_name(cfg).startswith(PREFIX[request.param.split("_")[0]])
    qctx.set("batched_cfg", cfg)
    yield request.param
    qctx.set("batched_cfg", -1)


@pytest.fixture(scope="module")
def small_batch():
    """24 matrices of the batched workload's distribution (sizes uniform in [32, 256], cond <= 1e3)."""
    sizes = qsynth.c4_sizes(count=24, seed=310)
    return [qsynth.round_f32(qsynth.c4_instance(b, sizes, seed0=310)) for b in range(24)]


@pytest.mark.parametrize("method,order", [("qhpi19", 19), ("qsai", 10), ("ns", 2)])
def test_batched_fixed_iterations_vs_oracle(qctx, small_batch, method, order):
    import paper_2605_01464_amd as q

    J = 3 if method != "ns" else 6
    alphas = [M.alpha_sigma(A) for A in small_batch]
    Xs, infos = q.solve_batched(qctx, [to_dev(A, "f32") for A in small_batch], method, order, scaling="given",
                                alphas=alphas, tol=0.0, max_iter=J, stop="dx_rel", check=False)
    for A, a, X, inf in zip(small_batch, alphas, Xs, infos):
        side = "left" if A.shape[1] > A.shape[2] else "right"
        ref = M.iterate(A, M.x0(A, a), method, order, side, J)[-1]
        assert inf["iters"] == J and inf["status"] == q.ENOTCONVERGED
        assert inf["alpha_used"] == a
        assert rel_fro(to_np(X), ref) <= 1e-4, (A.shape, rel_fro(to_np(X), ref))


def test_batched_converged_vs_pinv(qctx, small_batch):
    import paper_2605_01464_amd as q

    Xs, infos = q.solve_batched(qctx, [to_dev(A, "f32") for A in small_batch], "qhpi19", tol=1e-6, stop="guarded")
    errs = []
    for A, X, inf in zip(small_batch, Xs, infos):
        assert inf["status"] == q.OK and inf["reason"] in ("tol", "rise")
        f = M.features(A, 8)
        assert inf["sigma1_sq_est"] == pytest.approx(f["sigma1_sq"], rel=1e-9)
        errs.append(rel_fro(to_np(X), Q.pinv_svd(A)))
    assert max(errs) <= 1e-4, errs


def test_batched_equals_single_path_iterates(qctx, small_batch):
    """Same method, alpha and iteration count through the single-matrix path (other tile shapes and
    accumulation order): the two FP32 results agree to FP32 rounding."""
    import paper_2605_01464_amd as q

    As = [to_dev(A, "f32") for A in small_batch[:6]]
    alphas = [M.alpha_sigma(A) for A in small_batch[:6]]
    Xs, _ = q.solve_batched(qctx, As, "qhpi19", scaling="given", alphas=alphas, tol=0.0, max_iter=4, stop="dx_rel",
                            check=False)
    for Ad, a, Xb in zip(As, alphas, Xs):
        Xsingle, _ = q.solve(qctx, Ad, "qhpi19", scaling="given", alpha=a, tol=0.0, max_iter=4, stop="dx_rel",
                             precision="f32", check=False)
        assert rel_fro(to_np(Xb), to_np(Xsingle)) <= 1e-4


def test_batched_order_and_replay(qctx, small_batch):
    """Results do not depend on the position in the batch (bitwise), and a replayed graph with new
    inputs of the same shapes gives the new results."""
    import torch
    import paper_2605_01464_amd as q

    As = [to_dev(A, "f32") for A in small_batch[:8]]
    X1, _ = q.solve_batched(qctx, As, "qhpi19", tol=1e-6)
    perm = [3, 0, 7, 5, 1, 6, 2, 4]
    X2, _ = q.solve_batched(qctx, [As[i] for i in perm], "qhpi19", tol=1e-6)
    for k, i in enumerate(perm):
        assert torch.equal(X1[i], X2[k])
    # same shapes, new values -> graph replay
    As2 = [2.0 * a for a in As]
    X3, _ = q.solve_batched(qctx, As2, "qhpi19", tol=1e-6)
    for a2, x3 in zip(As2, X3):
        A2 = to_np(a2)
        assert rel_fro(to_np(x3), Q.pinv_svd(A2)) <= 1e-4


def test_batched_error_statuses(qctx, small_batch):
    import paper_2605_01464_amd as q

    As = [to_dev(A, "f32") for A in small_batch[:4]]
    bad = As[2].clone()
    bad[1, 3, 4] = float("nan")
    As[2] = bad
    Xs, infos = q.solve_batched(qctx, As, "qhpi19", tol=1e-6, check=False)
    assert infos[2]["status"] == q.ENONFINITE
    assert all(infos[i]["status"] == q.OK for i in (0, 1, 3))
    # invalid: FP64 storage, bad method
    st, _ = q.qpinv_solve_batched(qctx.handle, q.METHOD["qrapid"], 5, As[:1], [Xs[0]], 0, None, 1e-6, 50, 3)
    assert st == q.EINVAL


def test_batched_full_workload_sampled(qctx):
    """The 512-matrix batched workload; 48 sampled matrices checked against the FP64 pseudoinverse."""
    import paper_2605_01464_amd as q

    sizes = qsynth.c4_sizes()
    idx = np.random.default_rng(9).choice(512, 48, replace=False)
    mats = {}
    As = []
    for b in range(512):
        A = qsynth.round_f32(qsynth.c4_instance(b, sizes))
        if b in idx:
            mats[b] = A
        As.append(to_dev(A, "f32"))
    Xs, infos = q.solve_batched(qctx, As, "qhpi19", tol=1e-6, stop="guarded")
    assert all(inf["status"] == q.OK for inf in infos)
    errs = [rel_fro(to_np(Xs[b]), Q.pinv_svd(A)) for b, A in mats.items()]
    assert max(errs) <= 1e-4, (max(errs), float(np.median(errs)))


def test_sync_equals_queue_bitwise(qctx, small_batch, batched_form):
    """Both kernel forms run the same tile routine on the same operands: at a fixed number of updates the
    iterates agree bit for bit."""
    import torch

    import paper_2605_01464_amd as q

    if batched_form == "queue":
        pytest.skip("compares each phase-synchronous form with the queue form")
    As = [to_dev(A, "f32") for A in small_batch]
    alphas = [M.alpha_sigma(A) for A in small_batch]
    kw = dict(scaling="given", alphas=alphas, tol=0.0, max_iter=4, stop="dx_rel", check=False)
    Xs_sync, _ = q.solve_batched(qctx, As, "qhpi19", **kw)
    qctx.set("batched_cfg", FORMS["queue"])
    Xs_queue, _ = q.solve_batched(qctx, As, "qhpi19", **kw)
    for a, b in zip(Xs_sync, Xs_queue):
        assert torch.equal(a, b)


def test_sync_item_dealing_does_not_change_results(qctx, small_batch, batched_form):
    """Work items claimed from the phase counter (default) or dealt g, g + G, ...: every tile is computed by
    the same code on the same operands and the per-matrix sums run in tile order, so the converged
    iterates, iteration counts and statuses agree bit for bit."""
    import torch

    import paper_2605_01464_amd as q

    if batched_form == "queue":
        pytest.skip("item dealing exists in the phase-synchronous forms only")
    As = [to_dev(A, "f32") for A in small_batch]
    try:
        out = {}
        for dyn in (1, 0):
            qctx.set("batched_dynamic", dyn)
            Xs, infos = q.solve_batched(qctx, As, "qhpi19", tol=1e-6, stop="guarded")
            out[dyn] = (Xs, [(i["iters"], i["status"]) for i in infos])
    finally:
        qctx.set("batched_dynamic", 1)
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)


def test_batch_args_equal_list_arguments(qctx, small_batch, batched_form):
    """Descriptors marshalled once (BatchArgs) and reused: the same solve as the per-call tensor lists, bit for
    bit, on repeated calls; the outputs are the BatchArgs' own tensors."""
    import torch

    import paper_2605_01464_amd as q

    As = [to_dev(A, "f32") for A in small_batch]
    Xs_list, inf_list = q.solve_batched(qctx, As, "qhpi19", tol=1e-6, stop="guarded")
    args = q.BatchArgs(As)
    for _ in range(2):
        Xs_args, inf_args = q.solve_batched(qctx, args, "qhpi19", tol=1e-6, stop="guarded")
        assert all(x is y for x, y in zip(Xs_args, args.Xs))
        assert [(i["iters"], i["status"]) for i in inf_args] == [(i["iters"], i["status"]) for i in inf_list]
        for a, b in zip(Xs_args, Xs_list):
            assert torch.equal(a, b)
    with pytest.raises(ValueError):
        q.solve_batched(qctx, args, "qhpi19", Xs=Xs_list)
