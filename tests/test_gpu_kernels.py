"""GPU kernels vs the FP64 oracle: quaternion GEMM (every tile configuration), X_0, features."""
import numpy as np
import pytest

from conftest import to_dev, to_np
from oracle import quat as Q
from oracle import methods as M

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53

# (384, 384, 192) is a whole number of tiles of every configuration (the aligned, unchecked load path)
SHAPES = [(1, 1, 1), (7, 5, 3), (33, 65, 17), (100, 37, 129), (128, 128, 128), (130, 250, 70), (257, 129, 300),
          (384, 384, 192)]


def gemm_bound(A, B, C0, alpha, beta, gamma, u):
    """Elementwise rounding bound of fl(alpha A B + beta C0 + gamma I): every component of (A B)_ij is a
    sum of 4K signed plane products, so |error| <= gamma_{4K+3} (|alpha| S_ij + |beta| |C0| + |gamma|) with
    S_ij = sum_k (sum_q |A_q,ik|)(sum_r |B_r,kj|)."""
    K = A.shape[2]
    n = 4 * K + 3
    g = n * u / (1 - n * u)
    S = np.abs(A).sum(axis=0) @ np.abs(B).sum(axis=0)
    extra = abs(beta) * np.abs(C0) + abs(gamma)
    return g * (abs(alpha) * S[None] + extra) + 1e-300


def rng_planes(seed, m, n, dtype):
    A = np.random.default_rng(seed).standard_normal((4, m, n))
    return A.astype(np.float32).astype(np.float64) if dtype == "f32" else A


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shape", SHAPES)
def test_qgemm_every_config_within_rounding_bound(qctx, prec, shape):
    import paper_2605_01464_amd as q

    M_, N_, K_ = shape
    A = rng_planes(1, M_, K_, prec)
    B = rng_planes(2, K_, N_, prec)
    C0 = rng_planes(3, M_, N_, prec)
    alpha, beta, gamma = 0.75, -0.5, 2.0
    ref = alpha * Q.qmul(A, B) + beta * C0
    ref[0] += gamma * np.eye(M_, N_)
    u = U32 if prec == "f32" else U64
    bound = gemm_bound(A, B, C0, alpha, beta, gamma, u)
    gp = q.GEMM_PREC[prec]
    for cfg in range(q.qpinv_num_tile_configs(gp)):
        Ad, Bd = to_dev(A, prec), to_dev(B, prec)
        Cd = to_dev(C0, prec)
        q.qgemm(qctx, Ad, Bd, Cd, alpha, beta, gamma, gemm_prec=prec, cfg=cfg)
        err = np.abs(to_np(Cd) - ref)
        name = q.qpinv_tile_config_name(gp, cfg)
        assert np.all(err <= bound), (name, float(err.max()), float((err / bound).max()))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_qgemm_strided_views_and_ragged_ld(qctx, prec):
    import torch
    import paper_2605_01464_amd as q

    A = rng_planes(4, 45, 70, prec)
    B = rng_planes(5, 70, 33, prec)
    # operands embedded in larger buffers: ld and plane stride differ from cols / rows*cols
    big = torch.zeros((4, 50, 77), dtype=torch.float32 if prec == "f32" else torch.float64, device="cuda")
    big[:, :45, :70] = to_dev(A, prec)
    Av = big[:, :45, :70]
    Bd = to_dev(B, prec)
    Cbig = torch.zeros((4, 47, 35), dtype=big.dtype, device="cuda")
    Cv = Cbig[:, 1:46, 1:34]
    q.qgemm(qctx, Av, Bd, Cv, gemm_prec=prec)
    ref = Q.qmul(A, B)
    bound = gemm_bound(A, B, np.zeros_like(ref), 1.0, 0.0, 0.0, U32 if prec == "f32" else U64)
    assert np.all(np.abs(to_np(Cv) - ref) <= bound)
    # the padding around the view is untouched
    assert float(Cbig[:, 0, :].abs().max()) == 0.0 and float(Cbig[:, :, 0].abs().max()) == 0.0


def test_qgemm_empty_and_k_zero(qctx):
    import torch
    import paper_2605_01464_amd as q

    A = torch.zeros((4, 5, 0), device="cuda")
    B = torch.zeros((4, 0, 6), device="cuda")
    C = torch.full((4, 5, 6), 3.0, device="cuda")
    q.qgemm(qctx, A, B, C, alpha=1.0, beta=0.5, gamma=1.0)
    ref = np.full((4, 5, 6), 1.5)
    ref[0] += np.eye(5, 6)
    assert np.array_equal(to_np(C), ref)


def test_qgemm_bad_arguments(qctx):
    import torch
    import paper_2605_01464_amd as q

    A = torch.zeros((4, 5, 4), device="cuda")
    B = torch.zeros((4, 3, 6), device="cuda")
    C = torch.zeros((4, 5, 6), device="cuda")
    assert q.qpinv_qgemm(qctx.handle, q.GEMM_PREC["f32"], A, B, C) == q.EINVAL
    assert q.qpinv_qgemm(qctx.handle, q.GEMM_PREC["f64"], A, A.transpose(1, 2).contiguous(), C) == q.EINVAL


@pytest.mark.parametrize("src,dst", [("f64", "f64"), ("f32", "f32"), ("f32", "f64"), ("f64", "f32")])
def test_x0_bit_exact(qctx, src, dst):
    import paper_2605_01464_amd as q

    A = rng_planes(7, 70, 45, src)
    alpha = 0.0123
    X = q.x0(qctx, to_dev(A, src), alpha, out_dtype=to_dev(A[:, :1, :1], dst).dtype)
    ref = M.x0(A, alpha)
    if dst == "f32":
        ref = ref.astype(np.float32).astype(np.float64)
    assert np.array_equal(to_np(X), ref)


@pytest.mark.parametrize("shape", [(1, 1), (64, 48), (300, 77), (77, 300)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_features_match_oracle(qctx, shape, prec):
    import paper_2605_01464_amd as q

    A = rng_planes(8, *shape, prec)
    f = q.features(qctx, to_dev(A, prec), power_steps=6)
    o = M.features(A, 6)
    for k in ("fro", "norm1", "norminf"):
        assert f[k] == pytest.approx(o[k], rel=1e-12)
    assert f["sigma1_sq"] == pytest.approx(o["sigma1_sq"], rel=1e-10)
    assert (f["m"], f["n"]) == shape


def test_features_reject_nonfinite(qctx):
    import paper_2605_01464_amd as q

    A = rng_planes(9, 20, 10, "f64")
    A[2, 3, 4] = np.nan
    st, _ = q.qpinv_features(qctx.handle, to_dev(A, "f64"))
    assert st == q.ENONFINITE


@pytest.mark.parametrize("n", [2048, 4096])
def test_qgemm_square_relative_error_le_1e6(qctx, n):
    """Square FP32 quaternion product: relative Frobenius error vs the FP64 product of the same FP32
    inputs, on 24 sampled rows (the oracle computes those rows exactly), must be <= 1e-6."""
    import torch
    import paper_2605_01464_amd as q

    g = torch.Generator(device="cuda").manual_seed(400)
    A = torch.randn((4, n, n), device="cuda", generator=g)
    B = torch.randn((4, n, n), device="cuda", generator=g)
    C = q.qgemm(qctx, A, B)
    rows = np.random.default_rng(n).choice(n, 24, replace=False)
    Ah = A[:, rows, :].double().cpu().numpy()
    Bh = B.double().cpu().numpy()
    ref = Q.qmul(Ah, Bh)
    err = np.linalg.norm(C[:, rows, :].double().cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"n={n} rel err {err:.3e}")
    assert err <= 1e-6


@pytest.mark.parametrize("n", [2048, 4096])
def test_qgemm_bf16_full_size_sampled_rows(qctx, n):
    """Square BF16-operand product at the ladder's sizes in the configuration the library picks there
    (the staged form): relative Frobenius error vs the exact product of the BF16-rounded inputs, on 24
    sampled rows, within FP32 accumulation (<= 1e-6)."""
    import torch
    import paper_2605_01464_amd as q

    g = torch.Generator(device="cuda").manual_seed(410)
    A = torch.randn((4, n, n), device="cuda", generator=g)
    B = torch.randn((4, n, n), device="cuda", generator=g)
    C = q.qgemm(qctx, A, B, gemm_prec="bf16")
    rows = np.random.default_rng(n + 1).choice(n, 24, replace=False)
    ref = Q.qmul(round_bf16(A[:, rows, :].cpu().numpy()), round_bf16(B.cpu().numpy()))
    err = np.linalg.norm(C[:, rows, :].double().cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-6, err


def test_qgemm_bf16_beyond_the_staged_copy_limit(qctx):
    """A 16512 x 256 x 16384 BF16 product: 1032 output tiles of 64 x 64 select the staged form, whose copy
    of A would reach 2^31 bytes; the library computes it with the direct form instead (sampled rows
    against the exact product of the rounded inputs, within the random-walk scale u32 sqrt(4K) of FP32
    accumulation over 4K = 65536 terms)."""
    import torch
    import paper_2605_01464_amd as q

    M_, N_, K_ = 16512, 256, 16384
    assert 4 * M_ * K_ * 2 >= 2 ** 31 and ((M_ + 63) // 64) * ((N_ + 63) // 64) >= 1024
    g = torch.Generator(device="cuda").manual_seed(420)
    A = torch.randn((4, M_, K_), device="cuda", generator=g)
    B = torch.randn((4, K_, N_), device="cuda", generator=g)
    C = q.qgemm(qctx, A, B, gemm_prec="bf16")
    rows = np.random.default_rng(7).choice(M_, 8, replace=False)
    ref = Q.qmul(round_bf16(A[:, rows, :].cpu().numpy()), round_bf16(B.cpu().numpy()))
    err = np.linalg.norm(C[:, rows, :].double().cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 2.0 ** -24 * np.sqrt(4 * K_), err
    del A, B, C
    torch.cuda.empty_cache()


def round_bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_round_bf16_helper():
    assert round_bf16(np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5]))[0] == 1.0
    v = round_bf16(np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8]))
    assert v[0] == 1.0 and v[1] == 1.0 + 2 ** -6  # ties go to the even mantissa


def _bf16_cfgs(q, tag):
    gp = q.GEMM_PREC["bf16"]
    return [c for c in range(q.qpinv_num_tile_configs(gp)) if tag in q.qpinv_tile_config_name(gp, c)]


def test_qgemm_bf16_staged_equals_direct_and_regrows_its_stage(qctx):
    """The staged form (BF16 copies of the operands, zero-padded to whole tiles and K steps) with the
    16 x 16 x 32 MFMA computes the same MFMA sequence over k as the forms that round while staging:
    identical outputs, epilogue included.
    Products of growing and shrinking size reuse and regrow the context's stage buffer."""
    import paper_2605_01464_amd as q

    # (the 32 x 32 x 16 MFMA splits each 32-k step in two: its sums round differently, and the
    # every-configuration test bounds it instead)
    staged = [c for c in _bf16_cfgs(q, "_staged") if c in _bf16_cfgs(q, "mfma16x16x32")]
    direct = _bf16_cfgs(q, "_db")
    assert staged and direct
    for seed, (M_, N_, K_) in enumerate([(130, 250, 70), (1, 1, 1), (700, 520, 333), (257, 129, 300), (64, 64, 32),
                                         (96, 40, 0)]):
        A = rng_planes(80 + seed, M_, K_, "f32")
        B = rng_planes(90 + seed, K_, N_, "f32")
        C0 = rng_planes(100 + seed, M_, N_, "f32")
        outs = {}
        for cfg in staged + direct:
            Cd = to_dev(C0, "f32")
            q.qgemm(qctx, to_dev(A, "f32"), to_dev(B, "f32"), Cd, 0.5, -1.25, 1.0, gemm_prec="bf16", cfg=cfg)
            outs[cfg] = to_np(Cd)
        for cfg in staged:
            assert np.array_equal(outs[cfg], outs[direct[0]]), (M_, N_, K_, cfg)


@pytest.mark.parametrize("shape", SHAPES)
def test_qgemm_bf16_every_config(qctx, shape):
    """BF16-operand product = exact product of the BF16-rounded FP32 inputs up to FP32 accumulation."""
    import paper_2605_01464_amd as q

    M_, N_, K_ = shape
    A = rng_planes(21, M_, K_, "f32")
    B = rng_planes(22, K_, N_, "f32")
    C0 = rng_planes(23, M_, N_, "f32")
    alpha, beta, gamma = 0.75, -0.5, 2.0
    Ab, Bb = round_bf16(A), round_bf16(B)
    ref = alpha * Q.qmul(Ab, Bb) + beta * C0
    ref[0] += gamma * np.eye(M_, N_)
    bound = gemm_bound(Ab, Bb, C0, alpha, beta, gamma, U32)
    for cfg in range(q.qpinv_num_tile_configs(q.GEMM_PREC["bf16"])):
        Cd = to_dev(C0, "f32")
        q.qgemm(qctx, to_dev(A, "f32"), to_dev(B, "f32"), Cd, alpha, beta, gamma, gemm_prec="bf16", cfg=cfg)
        err = np.abs(to_np(Cd) - ref)
        name = q.qpinv_tile_config_name(q.GEMM_PREC["bf16"], cfg)
        assert np.all(err <= bound), (name, float(err.max()), float((err / bound).max()))


def split_bf16(x):
    """x = hi + lo + d with hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32), as float64."""
    hi = round_bf16(x)
    return hi, round_bf16((np.asarray(x, dtype=np.float64) - hi).astype(np.float32))


def test_split_bf16_helper():
    # BF16 keeps 8 significant bits: spacing 2^-7 above 1, 2^-16 at 2^-9
    x = np.array([1.0 + 2 ** -9 + 2 ** -20, -3.0, 1e-30, 1.0 + 2 ** -8 + 2 ** -20], dtype=np.float32).astype(np.float64)
    hi, lo = split_bf16(x)
    assert hi[0] == 1.0 and lo[0] == 2 ** -9 and hi[1] == -3.0 and lo[1] == 0.0
    assert hi[3] == 1.0 + 2 ** -7 and lo[3] == -(2 ** -8)  # x - hi = -2^-8 + 2^-20 keeps 8 bits of it
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))


@pytest.mark.parametrize("shape", SHAPES)
def test_qgemm_bf16x3_every_config(qctx, shape):
    """Three-product form: equal, up to FP32 accumulation over its 3 x 4K terms, to hi.hi + hi.lo + lo.hi of
    the split FP32 inputs, and within that plus 3 2^-16 S (the dropped lo.lo term and the split remainders)
    of the exact product; at least 30x closer to it than the one-product BF16 form on the larger shapes."""
    import paper_2605_01464_amd as q

    M_, N_, K_ = shape
    A = rng_planes(31, M_, K_, "f32")
    B = rng_planes(32, K_, N_, "f32")
    C0 = rng_planes(33, M_, N_, "f32")
    alpha, beta, gamma = 0.75, -0.5, 2.0
    (Ah, Al), (Bh, Bl) = split_bf16(A), split_bf16(B)
    A3, B3 = np.concatenate([Ah, Ah, Al], axis=2), np.concatenate([Bh, Bl, Bh], axis=1)
    ref3 = alpha * Q.qmul(A3, B3) + beta * C0
    ref3[0] += gamma * np.eye(M_, N_)
    bound3 = gemm_bound(A3, B3, C0, alpha, beta, gamma, U32)
    ref = alpha * Q.qmul(A, B) + beta * C0
    ref[0] += gamma * np.eye(M_, N_)
    S = np.abs(A).sum(axis=0) @ np.abs(B).sum(axis=0)
    bound = bound3 + 3.0 * 2.0 ** -16 * abs(alpha) * S[None]
    gp = q.GEMM_PREC["bf16x3"]
    assert q.qpinv_num_tile_configs(gp) >= 1
    Cb = to_dev(C0, "f32")
    q.qgemm(qctx, to_dev(A, "f32"), to_dev(B, "f32"), Cb, alpha, beta, gamma, gemm_prec="bf16")
    err_bf16 = np.abs(to_np(Cb) - ref).max()
    for cfg in range(q.qpinv_num_tile_configs(gp)):
        Cd = to_dev(C0, "f32")
        q.qgemm(qctx, to_dev(A, "f32"), to_dev(B, "f32"), Cd, alpha, beta, gamma, gemm_prec="bf16x3", cfg=cfg)
        out = to_np(Cd)
        name = q.qpinv_tile_config_name(gp, cfg)
        e3 = np.abs(out - ref3)
        assert np.all(e3 <= bound3), (name, float(e3.max()), float((e3 / bound3).max()))
        e = np.abs(out - ref)
        assert np.all(e <= bound), (name, float(e.max()), float((e / bound).max()))
        if K_ >= 64:
            assert e.max() * 30 <= err_bf16, (name, float(e.max()), float(err_bf16))
