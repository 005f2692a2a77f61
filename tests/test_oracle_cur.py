"""CUR approximation and completion of Section 5.1 (oracle), pinned by exact reconstruction of low-rank
matrices (both couplings), the optimality conditions of U = C^+ A R^+, and closed-form PSNR / merge cases."""
import numpy as np

import qsynth
from oracle import cur
from oracle import quat as Q


def _low_rank(seed, m, n, k):
    return qsynth.small_spectral_instance(seed, m, n, np.linspace(3.0, 1.0, k))["A"]


def test_exact_low_rank_is_reconstructed_by_both_couplings():
    """rank(C) = rank(R) = rank(A) = k: C U R = A for U = C^+ A R^+ and for U = W^+."""
    A = _low_rank(21, 60, 50, 8)
    rng = np.random.default_rng(22)
    rows = np.sort(rng.choice(60, 12, replace=False))
    cols = np.sort(rng.choice(50, 12, replace=False))
    X, U = cur.reconstruct(A, rows, cols)
    assert U.shape == (4, 12, 12)
    assert Q.fro(X - A) <= 1e-10 * Q.fro(A)
    assert Q.fro(cur.reconstruct_cross(A, rows, cols) - A) <= 1e-9 * Q.fro(A)


def test_coupling_satisfies_the_optimality_conditions():
    """U = C^+ A R^+ minimises ||A - C U R||_F: the gradient C^H (A - C U R) R^H vanishes, and a perturbed
    coupling is worse."""
    A = qsynth.gaussian(23, 40, 30)
    rng = np.random.default_rng(24)
    rows = np.sort(rng.choice(40, 10, replace=False))
    cols = np.sort(rng.choice(30, 10, replace=False))
    X, U = cur.reconstruct(A, rows, cols)
    C, R, _ = cur.factors(A, rows, cols)
    g = Q.qmul(Q.qmul(Q.qH(C), A - X), Q.qH(R))
    assert Q.fro(g) <= 1e-10 * Q.fro(C) * Q.fro(A) * Q.fro(R)
    E = Q.qmul(Q.qmul(C, U + 1e-3 * qsynth.gaussian(25, 10, 10)), R)
    assert Q.fro(A - E) > Q.fro(A - X)


def test_merge_and_psnr_closed_forms():
    M = qsynth.gaussian(26, 5, 6)
    X = qsynth.gaussian(27, 5, 6)
    mask = (np.arange(30).reshape(5, 6) % 3 == 0).astype(np.uint8)
    Y = cur.merge(M, mask, X)
    assert np.array_equal(Y[:, mask == 1], M[:, mask == 1]) and np.array_equal(Y[:, mask == 0], X[:, mask == 0])
    ref = np.zeros((4, 5, 6))
    assert abs(cur.psnr(ref + 0.1, ref) - 20.0) < 1e-12


def test_completion_keeps_observed_pixels_and_improves():
    d = qsynth.cur_image_instance(96, 128, terms=8, rank=16, seed=28)
    img, mask = d["image"], d["mask"]
    Xs = cur.complete(img, mask, d["rows"], d["cols"], 4)
    first, _ = cur.reconstruct(cur.merge(img, mask, np.zeros_like(img)), d["rows"], d["cols"])
    assert np.array_equal(Xs[0], first)
    p = [cur.psnr(X, img) for X in Xs]
    assert all(b > a for a, b in zip(p, p[1:])), p
    assert p[0] > cur.psnr(cur.merge(img, mask, np.zeros_like(img)), img)
