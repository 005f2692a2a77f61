"""Tile configurations whose workgroups walk several output tiles (c workgroups per compute unit)
against the same tile shape with one tile per workgroup, and against the FP64 oracle; the persisted
tile choices (tune cache) of a context."""
import numpy as np
import pytest

from conftest import to_dev, to_np
from oracle import quat as Q
from test_gpu_kernels import U32, U64, gemm_bound, rng_planes, round_bf16

pytestmark = pytest.mark.gpu

PRECS = ["f32", "bf16"]  # the precisions whose tables hold walking configurations


def walking_configs(q, gp):
    """(per-CU configuration, the one-tile-per-workgroup configuration of the same kernel)."""
    names = {q.qpinv_tile_config_name(gp, c): c for c in range(q.qpinv_num_tile_configs(gp))}
    return [(c, names[n.rsplit("_cu", 1)[0]]) for n, c in names.items() if "_cu" in n]


@pytest.mark.parametrize("prec", PRECS)
def test_walking_configs_exist(qctx, prec):
    import paper_2605_01464_amd as q

    assert walking_configs(q, q.GEMM_PREC[prec])


@pytest.mark.parametrize("prec", PRECS)
def test_qgemm_walking_tiles_within_bound_and_equal_to_one_tile_per_workgroup(qctx, prec):
    """1500 x 1400 outputs: 2068 tiles of 32 x 32 and 528 of 64 x 64, more than any per-CU grid holds."""
    import paper_2605_01464_amd as q

    M_, N_, K_ = 1500, 1400, 40
    store = "f64" if prec == "f64" else "f32"
    A = rng_planes(31, M_, K_, store)
    B = rng_planes(32, K_, N_, store)
    C0 = rng_planes(33, M_, N_, store)
    alpha, beta, gamma = 0.75, -0.5, 2.0
    Ar, Br = (round_bf16(A), round_bf16(B)) if prec == "bf16" else (A, B)
    ref = alpha * Q.qmul(Ar, Br) + beta * C0
    ref[0] += gamma * np.eye(M_, N_)
    bound = gemm_bound(Ar, Br, C0, alpha, beta, gamma, U64 if prec == "f64" else U32)
    gp = q.GEMM_PREC[prec]
    Ad, Bd = to_dev(A, store), to_dev(B, store)
    for cfg, base in walking_configs(q, gp):
        outs = []
        for c in (cfg, base):
            Cd = to_dev(C0, store)
            q.qgemm(qctx, Ad, Bd, Cd, alpha, beta, gamma, gemm_prec=prec, cfg=c)
            outs.append(to_np(Cd))
        name = q.qpinv_tile_config_name(gp, cfg)
        err = np.abs(outs[0] - ref)
        assert np.all(err <= bound), (name, float((err / bound).max()))
        assert np.array_equal(outs[0], outs[1]), name  # same tiles, same arithmetic


@pytest.mark.parametrize("prec", PRECS)
def test_step_reduction_with_walking_tiles(qctx, prec):
    """One QHPI19 update (7 products with fused epilogues and the change reduction) with every product
    forced to a walking configuration equals the update with one tile per workgroup: the iterate
    bitwise, the change norm up to the order of the per-workgroup partial sums."""
    import torch

    import paper_2605_01464_amd as q

    store = "f64" if prec == "f64" else "f32"
    A = rng_planes(41, 1600, 1500, store)
    Ad = to_dev(A, store)
    alpha = 1.0 / float(np.sum(A * A))
    X0 = q.x0(qctx, Ad, alpha)
    gp = q.GEMM_PREC[prec]
    key = {"f64": "gemm_cfg_f64", "f32": "gemm_cfg_f32", "bf16": "gemm_cfg_bf16"}[prec]
    try:
        for cfg, base in walking_configs(q, gp):
            res = []
            for c in (cfg, base):
                qctx.set(key, c)
                out, dx = q.step(qctx, Ad, X0, method="qhpi19", gemm_prec=prec)
                torch.cuda.synchronize()
                res.append((to_np(out), dx))
            name = q.qpinv_tile_config_name(gp, cfg)
            assert np.array_equal(res[0][0], res[1][0]), name
            for a, b in zip(res[0][1], res[1][1]):  # (||X_1 - X_0||_F, ||X_1||_F)
                assert abs(a - b) <= 1e-12 * abs(b), (name, res[0][1], res[1][1])
    finally:
        qctx.set(key, -1)


def test_tune_cache_round_trip(tmp_path):
    """Tile choices tuned on one context, saved to a file and loaded into a fresh context, which then holds the
    same choices (its own save writes the same file); a file for another device applies nothing, an entry
    naming an unknown configuration is skipped, and a malformed file is refused with nothing applied."""
    import paper_2605_01464_amd as q

    path, path2 = tmp_path / "tune.txt", tmp_path / "tune2.txt"
    with q.Context(0) as a:
        c32, _ = q.qpinv_autotune(a.handle, q.GEMM_PREC["f32"], 96, 80, 64)
        c64, _ = q.qpinv_autotune(a.handle, q.GEMM_PREC["f64"], 33, 17, 29)
        assert c32 >= 0 and c64 >= 0
        assert a.save_tuning(path) == 2
    text = path.read_text()
    lines = text.splitlines()
    assert lines[0].startswith("qpinv-tune 1 ") and len(lines) == 3
    assert f"gemm 1 96 80 64 {q.qpinv_tile_config_name(q.GEMM_PREC['f32'], c32)}" in lines
    assert f"gemm 0 33 17 29 {q.qpinv_tile_config_name(q.GEMM_PREC['f64'], c64)}" in lines
    with q.Context(0) as b:
        assert b.load_tuning(path) == 2
        assert b.save_tuning(path2) == 2
        assert path2.read_text() == text
        other = tmp_path / "other.txt"
        other.write_text("qpinv-tune 1 gfx000:1cu\n" + "\n".join(lines[1:]) + "\n")
        assert b.load_tuning(other) == 0
        unknown = tmp_path / "unknown.txt"
        unknown.write_text(text + "gemm 1 5 5 5 no_such_config\n")
        assert b.load_tuning(unknown) == 2
        bad = tmp_path / "bad.txt"
        bad.write_text(lines[0] + "\ngemm 1 7 7 7 " + q.qpinv_tile_config_name(q.GEMM_PREC["f32"], 0) + "\ngemm 1 x\n")
        with pytest.raises(q.QpinvError):
            b.load_tuning(bad)
        assert b.save_tuning(path2) == 2  # nothing of the malformed file was applied
        with pytest.raises(q.QpinvError):
            b.load_tuning(tmp_path / "missing.txt")
