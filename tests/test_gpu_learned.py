"""Learned initial scaling on the GPU: network kernels vs the FP64 reference, labels vs the spectral
model and vs actual solves, and what a trained network gains over the classical alpha."""
import numpy as np
import pytest

import qsynth
from conftest import rel_fro, to_dev, to_np
from oracle import methods as M
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


def random_raw(rng, n):
    """Plausible raw feature rows (s1sq, s1sq_prev, fro, norm1, norminf, m, n)."""
    m = rng.integers(64, 512, n).astype(float)
    k = rng.integers(64, 512, n).astype(float)
    s1 = 10 ** rng.uniform(-2, 2, n)
    prev = s1 * rng.uniform(0.8, 1.0, n)
    fro = np.sqrt(s1 * rng.uniform(1.0, np.minimum(m, k)))
    n1 = np.sqrt(s1) * rng.uniform(1.0, 3.0, n) * np.sqrt(m) * 0.5
    ni = np.sqrt(s1) * rng.uniform(1.0, 3.0, n) * np.sqrt(k) * 0.5
    return np.stack([s1, prev, fro, n1, ni, m, k], axis=1)


def set_params(q, ctx, rng):
    theta = (0.2 * rng.standard_normal(OM.NPARAM)).astype(np.float32)
    mean = rng.standard_normal(10).astype(np.float32)
    std = rng.uniform(0.5, 2.0, 10).astype(np.float32)
    q._err(q.qpinv_mlp_set_params(ctx.handle, list(np.concatenate([theta, mean, std]))), "set")
    return theta.astype(np.float64), mean.astype(np.float64), std.astype(np.float64)


def test_gradient_matches_fp64_backprop(qctx):
    import torch
    import paper_2605_01464_amd as q

    rng = np.random.default_rng(1)
    theta, mean, std = set_params(q, qctx, rng)
    raw = random_raw(rng, 200)
    tgt = rng.standard_normal(200)
    grad = torch.empty(OM.NPARAM, dtype=torch.float32, device="cuda")
    st, loss = q.qpinv_mlp_gradient(qctx.handle, torch.from_numpy(raw).cuda(), torch.from_numpy(tgt).cuda(), grad)
    assert st == q.OK
    Z = (OM.transform(raw) - mean) / std
    lo, go = OM.loss_and_grad(theta, Z, tgt)
    g = grad.double().cpu().numpy()
    assert loss == pytest.approx(lo, rel=1e-4)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_predict_matches_fp64_forward(qctx):
    import torch
    import paper_2605_01464_amd as q

    rng = np.random.default_rng(2)
    theta, mean, std = set_params(q, qctx, rng)
    raw = random_raw(rng, 300)
    mu = torch.empty(300, dtype=torch.float64, device="cuda")
    assert q.qpinv_mlp_predict(qctx.handle, torch.from_numpy(raw).cuda(), mu) == q.OK
    y, _ = OM.forward(theta, (OM.transform(raw) - mean) / std)
    np.testing.assert_allclose(mu.cpu().numpy(), np.exp(y), rtol=2e-5)


def test_train_step_is_adam(qctx):
    """One GPU training step equals the FP64 Adam update of the FP64 gradient (to FP32 rounding)."""
    import torch
    import paper_2605_01464_amd as q

    rng = np.random.default_rng(3)
    theta, mean, std = set_params(q, qctx, rng)
    raw = random_raw(rng, 64)
    tgt = rng.standard_normal(64)
    st, _ = q.qpinv_mlp_train_step(qctx.handle, torch.from_numpy(raw).cuda(), torch.from_numpy(tgt).cuda(), None, 64,
                                   1e-3)
    assert st == q.OK
    _, vals = q.qpinv_mlp_get_params(qctx.handle)
    th_gpu = np.asarray(vals[:OM.NPARAM], dtype=np.float64)
    _, g = OM.loss_and_grad(theta, (OM.transform(raw) - mean) / std, tgt)
    th_ref, _, _ = OM.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), g, 1, lr=1e-3)
    # the first Adam step moves each weight by ~lr * sign(g); compare the displacement
    np.testing.assert_allclose(th_gpu - theta, th_ref - theta, atol=2e-6)


def _oracle_label(s, s1sq_est, method, order, tol, ngrid=64, lo=0.05, hi=1.95, target=1.8):
    smax2 = float(np.max(s)) ** 2
    mus = lo * (hi / lo) ** (np.arange(ngrid) / (ngrid - 1))
    J = np.array([M.spectral_iterations(s, mu / smax2, method, order, tol, max_iter=64) for mu in mus])
    best = J.min()
    runs, cur0, curlen, best_run = [], -1, 0, (0, 0)
    for k in range(ngrid):
        if J[k] == best:
            cur0 = k if curlen == 0 else cur0
            curlen += 1
            if curlen > best_run[1]:
                best_run = (cur0, curlen)
        else:
            curlen = 0
    mu_a = lo * (hi / lo) ** (best_run[0] / (ngrid - 1))
    mu_b = lo * (hi / lo) ** ((best_run[0] + best_run[1] - 1) / (ngrid - 1))
    mu_star = min(max(target, mu_a), mu_b)
    jc = M.spectral_iterations(s, 1.0 / s1sq_est, method, order, tol, max_iter=64)
    return mu_star / smax2 * s1sq_est, best, jc


@pytest.mark.parametrize("method,order", [("qhpi19", 19), ("ns", 2), ("qrapid", 5)])
def test_labels_match_spectral_model(qctx, method, order):
    import torch
    import paper_2605_01464_amd as q

    specs = [qsynth.c5_spectrum(s, 150, 110, fam) for s, fam in zip(range(6), qsynth.C5_FAMILIES * 2)]
    s1e = [float(s[0] ** 2 * 0.97) for s in specs]
    offs = np.concatenate([[0], np.cumsum([len(s) for s in specs])]).astype(np.int32)
    mu = torch.empty(6, dtype=torch.float64, device="cuda")
    jb = torch.empty(6, dtype=torch.int32, device="cuda")
    jc = torch.empty(6, dtype=torch.int32, device="cuda")
    st = q.qpinv_spectral_labels(qctx.handle, q.METHOD[method], order, torch.from_numpy(np.concatenate(specs)).cuda(),
                                 torch.from_numpy(offs).cuda(), torch.tensor(s1e, dtype=torch.float64).cuda(), 1e-10,
                                 64, 64, 0.05, 1.95, 1.8, mu, jb, jc)
    assert st == q.OK
    for b, s in enumerate(specs):
        mo, bo, co = _oracle_label(s, s1e[b], method, order, 1e-10)
        assert int(jb[b]) == bo and int(jc[b]) == min(co, 65)
        assert float(mu[b]) == pytest.approx(mo, rel=1e-12)


def test_label_counts_equal_gpu_fp64_solves(qctx):
    """The spectral iteration count behind the labels is what an FP64 QHPI19 solve with that alpha actually
    takes (+-1): 12 matrices of 256..512 (4 per spectrum family) at three points of the label grid."""
    import paper_2605_01464_amd as q

    seen = {f: 0 for f in qsynth.C5_FAMILIES}
    seed = 70_000
    while min(seen.values()) < 4:
        d = qsynth.c5_sample(seed, size_range=(256, 512))
        seed += 1
        if seen[d["family"]] >= 4:
            continue
        seen[d["family"]] += 1
        s = d["s"]
        Ad = to_dev(d["A"], "f64")
        for mu in (0.6, 1.0, 1.6):
            alpha = mu / s[0] ** 2
            J = M.spectral_iterations(s, alpha, "qhpi19", 19, 1e-10)
            _, info = q.solve(qctx, Ad, "qhpi19", scaling="given", alpha=alpha, tol=1e-10, stop="e1_rel",
                              precision="f64", max_iter=60)
            assert abs(info["iters"] - J) <= 1, (seed, d["family"], mu, info["iters"], J)


@pytest.mark.parametrize("seed", [2_000_000, 2_000_001, 2_000_008])  # geometric, clustered, low rank + noise
def test_eval_size_parity_vs_oracle(qctx, seed):
    """Held-out 1024 x 768 evaluation matrices, FP64 QHPI19 to ||AXA - A||_F / ||A||_F <= 1e-10 from the shipped
    network's alpha and from the classical alpha: each X against the oracle's solve from the same alpha, same
    stop rule and side, <= 1e-9, with the same update count."""
    import sys

    import paper_2605_01464_amd as q
    from paper_2605_01464_amd import learned as L

    d = qsynth.c5_sample(seed, shape=(1024, 768))
    L.load(qctx)
    Ad = to_dev(d["A"], "f64")
    for scaling in ("learned", "power"):
        X, info = q.solve(qctx, Ad, "qhpi19", scaling=scaling, tol=1e-10, stop="e1_rel", precision="f64", max_iter=60)
        assert info["status"] == q.OK and info["reason"] == "tol", info
        print(f"{d['family']} {scaling}: mu {info['mu_used']:.3f}, {info['iters']} updates; oracle", file=sys.stderr,
              flush=True)
        ro = M.solve(d["A"], "qhpi19", alpha=info["alpha_used"], tol=1e-10, stop="e1_rel", side="left", max_iter=60)
        assert info["iters"] == ro.iters, (info["iters"], ro.iters)
        assert rel_fro(to_np(X), ro.X) <= 1e-9


def test_trained_network_gain(qctx):
    """Train on 800 matrices (64..192) and evaluate on 40 held-out 160 x 128 matrices: the learned alpha
    needs no more iterations on average than the classical 1/sigma1_est^2 and than 1/||A||_F^2."""
    import paper_2605_01464_amd as q
    from paper_2605_01464_amd import learned as L

    train = L.build_set(qctx, range(50_000, 50_800), size_range=(64, 192))
    hist = L.train(qctx, train, epochs=40, batch=128)
    assert hist[-1] < hist[0]
    ev = L.build_set(qctx, range(60_000, 60_040), shape=(160, 128), keep=True)
    res, arms = L.evaluate(qctx, ev["mats"], ev)
    print(res)
    assert res["learned"]["mean_iters"] <= res["classical"]["mean_iters"] + 1e-9
    assert res["learned"]["mean_iters"] <= res["frobenius"]["mean_iters"]
    assert res["best"]["mean_iters"] <= res["learned"]["mean_iters"] + 1.0


def test_shipped_network_pays_at_eval_size(qctx):
    """The shipped network (trained on 20k matrices of 64..512) on the first 64 held-out 1024 x 768 evaluation
    matrices, FP64 QHPI19 to E1_rel <= 1e-10, arms interleaved per matrix: fewer updates on average than the
    classical alpha = 1/sigma1_est^2, and less wall time per solve (features, network and updates included)."""
    import paper_2605_01464_amd as q
    from paper_2605_01464_amd import learned as L

    L.load(qctx)
    ev = L.build_set(qctx, range(2_000_000, 2_000_064), shape=(1024, 768), keep=True)
    L.evaluate(qctx, ev["mats"][:4], ev)  # warm-up
    res, _ = L.evaluate(qctx, ev["mats"], ev)
    print({k: res[k] for k in ("learned", "classical", "best")})
    assert res["learned_fallbacks"] == 0
    assert res["learned"]["mean_iters"] < res["classical"]["mean_iters"]
    assert res["learned"]["mean_ms"] < res["classical"]["mean_ms"]


@pytest.mark.parametrize("stop", ["e1_rel", "guarded"])
def test_learned_guard_falls_back(qctx, stop):
    """A network that always answers mu = 1.9 on a matrix whose power estimate is low enough that
    1.9 / sigma1_est^2 > 2 / sigma_1^2: under the E1 stop the divergence restarts the solve from the classical
    alpha, under the guarded stop the ||I - X_0 A||_2 > 1 estimate does before the first update."""
    import paper_2605_01464_amd as q

    theta = np.zeros(OM.NPARAM, dtype=np.float32)
    theta[-1] = np.log(1.9)  # b3: constant output
    q._err(q.qpinv_mlp_set_params(qctx.handle, list(np.concatenate([theta, np.zeros(10), np.ones(10)]))), "set")
    # 40 singular values spread over [0.6, 1]: three power steps reach only ~0.85 sigma_1^2, so
    # 1.9 / sigma1_est^2 > 2 / sigma_1^2 while the classical 1 / sigma1_est^2 stays admissible
    s = np.linspace(1.0, 0.6, 40)
    inst = qsynth.small_spectral_instance(21, 90, 70, s)
    qctx.set("power_steps", 3)
    try:
        X, info = q.solve(qctx, to_dev(inst["A"], "f64"), "qhpi19", scaling="learned", tol=1e-10, stop=stop,
                          precision="f64")
        qctx.set("small_path", 0)  # the learned solve runs product by product: compare with the same path
        Xc, ic = q.solve(qctx, to_dev(inst["A"], "f64"), "qhpi19", scaling="power", tol=1e-10, stop=stop,
                         precision="f64")
    finally:
        qctx.set("power_steps", 8)
        qctx.set("small_path", 1)
    assert 1.9 / info["sigma1_sq_est"] > 2.0 / s[0] ** 2  # the network's alpha lies outside Theorem 1's interval
    assert info["fallback_used"] == 1 and info["reason"] in (("tol",) if stop == "e1_rel" else ("tol", "rise"))
    assert info["alpha_used"] == pytest.approx(1.0 / info["sigma1_sq_est"])
    assert ic["iters"] == info["iters"] and rel_fro(to_np(X), to_np(Xc)) == 0.0


def test_learned_restarts_at_max_iter(qctx):
    """A learned solve that reaches max_iter without meeting its test starts over from the classical alpha (a
    constant network answering mu = 0.05 on a flat spectrum 1 .. 0.9, where the clamp's lower end is 0.016:
    3 updates against the classical alpha's 1 by the spectral model, with max_iter = 1)."""
    import paper_2605_01464_amd as q

    theta = np.zeros(OM.NPARAM, dtype=np.float32)
    theta[-1] = np.log(0.05)
    q._err(q.qpinv_mlp_set_params(qctx.handle, list(np.concatenate([theta, np.zeros(10), np.ones(10)]))), "set")
    inst = qsynth.small_spectral_instance(22, 90, 70, np.linspace(1.0, 0.9, 70))
    Ad = to_dev(inst["A"], "f64")
    qctx.set("small_path", 0)  # the learned solve runs product by product: compare with the same path
    try:
        Xc, ic = q.solve(qctx, Ad, "qhpi19", scaling="power", tol=1e-10, stop="e1_rel", precision="f64", max_iter=40)
    finally:
        qctx.set("small_path", 1)
    X, info = q.solve(qctx, Ad, "qhpi19", scaling="learned", tol=1e-10, stop="e1_rel", precision="f64",
                      max_iter=ic["iters"])
    assert info["fallback_used"] == 1 and info["status"] == q.OK and info["reason"] == "tol", info
    assert info["iters"] == ic["iters"] and rel_fro(to_np(X), to_np(Xc)) == 0.0
