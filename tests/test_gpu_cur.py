"""CUR image completion of Section 5.1 on the GPU (submatrix gather, masked merge, two pseudoinverse
solves and four quaternion products per reconstruction) vs the FP64 oracle.

Tolerances (FP64 path): the pseudoinverses stop at the guarded rule with tol 1e-12, so each is within
~kappa * 1e-12 of the SVD definition (kappa <= 1e3 for these factors); the reconstruction inherits that
relative error, and a few completion steps add it a few times: 1e-7 relative."""
import numpy as np
import pytest

import qsynth
from conftest import to_dev, to_np
from oracle import cur
from oracle import quat as Q

pytestmark = pytest.mark.gpu


def _idx(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_submatrix_gathers_exactly(qctx, prec):
    import paper_2605_01464_amd as q

    A = qsynth.gaussian(31, 70, 90)
    rows = np.array([5, 0, 69, 33, 33, 12], dtype=np.int32)
    cols = np.array([89, 1, 2, 40, 3], dtype=np.int32)
    Ad = to_dev(A, prec)
    Ah = to_np(Ad)
    B = to_np(q.submatrix(qctx, Ad, _idx(rows), _idx(cols)))
    assert np.array_equal(B, Ah[:, rows][:, :, cols])
    assert np.array_equal(to_np(q.submatrix(qctx, Ad, None, _idx(cols))), Ah[:, :, cols])
    assert np.array_equal(to_np(q.submatrix(qctx, Ad, _idx(rows), None)), Ah[:, rows, :])
    bad = to_np(q.submatrix(qctx, Ad, _idx([1, 70, -1]), _idx([0, 1])))
    assert np.array_equal(bad[:, 0], Ah[:, 1][:, [0, 1]]) and np.isnan(bad[:, 1:]).all()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_masked_merge_exact_and_in_place(qctx, prec):
    import torch

    import paper_2605_01464_amd as q

    M = to_dev(qsynth.gaussian(32, 33, 47), prec)
    X = to_dev(qsynth.gaussian(33, 33, 47), prec)
    mask_h = (np.random.default_rng(34).uniform(size=(33, 47)) < 0.3).astype(np.uint8)
    mask = torch.from_numpy(mask_h).cuda()
    ref = np.where(mask_h[None] == 1, to_np(M), to_np(X))
    assert np.array_equal(to_np(q.masked_merge(qctx, M, mask, X)), ref)
    q.masked_merge(qctx, M, mask, X, out=X)  # Y aliases X
    assert np.array_equal(to_np(X), ref)


def test_cur_reconstruct_low_rank_and_general(qctx):
    import paper_2605_01464_amd as q

    A = qsynth.small_spectral_instance(35, 120, 90, np.linspace(3.0, 1.0, 10))["A"]
    rng = np.random.default_rng(36)
    rows = np.sort(rng.choice(120, 16, replace=False))
    cols = np.sort(rng.choice(90, 16, replace=False))
    X, U, infos = q.cur_reconstruct(qctx, to_dev(A, "f64"), _idx(rows), _idx(cols), tol=1e-12)
    assert Q.fro(to_np(X) - A) <= 1e-8 * Q.fro(A)
    G = qsynth.gaussian(37, 120, 90)
    Xg, Ug, _ = q.cur_reconstruct(qctx, to_dev(G, "f64"), _idx(rows), _idx(cols), tol=1e-12)
    Xo, Uo = cur.reconstruct(G, rows, cols)
    assert Q.fro(to_np(Ug) - Uo) <= 1e-7 * Q.fro(Uo)
    assert Q.fro(to_np(Xg) - Xo) <= 1e-7 * Q.fro(Xo)


def test_cur_completion_matches_oracle(qctx):
    import torch

    import paper_2605_01464_amd as q

    d = qsynth.cur_image_instance(96, 128, terms=8, rank=16, seed=38)
    img, mask = d["image"], d["mask"]
    ref = cur.complete(img, mask, d["rows"], d["cols"], 3)
    got = []
    q.cur_complete(qctx, to_dev(img, "f64"), torch.from_numpy(mask).cuda(), _idx(d["rows"]), _idx(d["cols"]),
                   iters=3, tol=1e-12, on_iter=lambda t, X: got.append(to_np(X)))
    assert len(got) == 3
    for a, b in zip(got, ref):
        assert Q.fro(a - b) <= 1e-7 * Q.fro(b)
    assert cur.psnr(got[-1], img) > cur.psnr(got[0], img)
