"""Tile configurations whose workgroups walk several output tiles (c workgroups per compute unit)
against the same tile shape with one tile per workgroup, and against the FP64 oracle."""
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
