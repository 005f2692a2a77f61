"""Global quaternion FOM / GMRES (Section 3.5, Example 4), oracle side, pinned by the definitions they
restate: the inner product Re tr(X^H Y), the Arnoldi relation and orthonormality of the basis, the
least-squares residual of GMRES, the Galerkin condition of FOM, and exact solves of small systems."""
import numpy as np
import pytest

import qsynth
from oracle import krylov as K
from oracle import methods as M
from oracle import quat as Q


def _small(m=2, grid=(3, 4), seed=701):
    return qsynth.krylov_instance(m, grid=grid, seed=seed)


def test_inner_product_is_real_trace():
    X = qsynth.gaussian(41, 7, 3)
    Y = qsynth.gaussian(42, 7, 3)
    assert abs(K.inner(X, Y) - np.trace(Q.qmul(Q.qH(X), Y)[0])) <= 1e-12 * Q.fro(X) * Q.fro(Y)
    assert np.allclose(Q.qmul(Q.qH(X), Y)[0].trace(), K.inner(Y, X))


@pytest.mark.parametrize("method", ["gmres", "fom"])
def test_arnoldi_relation_and_orthonormal_basis(method):
    d = _small(3, grid=(4, 5))
    r = K.solve(d["A"], d["B"], method, tol=0.0, max_iter=15)
    V, H, k = r["V"], r["H"], r["iters"]
    assert k == 15 and len(V) == 16
    G = np.array([[K.inner(a, b) for b in V] for a in V])
    assert np.max(np.abs(G - np.eye(len(V)))) <= 1e-10
    for j in range(k):
        lhs = Q.qmul(d["A"], V[j])
        rhs = sum(H[i, j] * V[i] for i in range(j + 2))
        assert Q.fro(lhs - rhs) <= 1e-11 * Q.fro(lhs)


def test_gmres_residual_is_the_least_squares_minimum():
    d = _small(2, grid=(4, 5))
    r = K.solve(d["A"], d["B"], "gmres", tol=0.0, max_iter=12)
    for k in range(1, 13):
        Hk = r["H"][: k + 1, :k]
        e = r["beta"] * np.eye(k + 1)[:, 0]
        y = np.linalg.lstsq(Hk, e, rcond=None)[0]
        assert abs(np.linalg.norm(e - Hk @ y) / r["beta"] - r["history"][k - 1]) <= 1e-12
    assert abs(r["true_rr"] - r["history"][-1]) <= 1e-10


def test_fom_residual_is_orthogonal_to_the_basis():
    d = _small(2, grid=(4, 5))
    r = K.solve(d["A"], d["B"], "fom", tol=0.0, max_iter=10)
    R = d["B"] - Q.qmul(d["A"], r["X"])
    for Vi in r["V"][:10]:
        assert abs(K.inner(Vi, R)) <= 1e-10 * Q.fro(R)
    assert abs(r["true_rr"] - r["history"][-1]) <= 1e-8


@pytest.mark.parametrize("method", ["gmres", "fom"])
def test_small_system_is_solved(method):
    d = _small(2)
    r = K.solve(d["A"], d["B"], method, tol=1e-12, max_iter=400)
    X = Q.from_cadj(np.linalg.solve(Q.cadj(d["A"]), Q.cadj(d["B"])))
    assert r["converged"] and r["true_rr"] <= 1e-12
    assert Q.fro(r["X"] - X) <= 1e-8 * Q.fro(X)


def test_preconditioned_run_stops_on_the_original_residual():
    d = _small(2, grid=(5, 6))
    A = d["A"]
    P = M.x0(A, M.alpha_sigma(A))
    for _ in range(3):
        P = M.step(A, P, "qsai")
    plain = K.solve(A, d["B"], "gmres", tol=1e-8, max_iter=800)
    pre = K.solve(A, d["B"], "gmres", M=P, tol=1e-8, max_iter=800)
    assert pre["true_rr"] <= 1e-8 and plain["true_rr"] <= 1e-8
    assert pre["iters"] < plain["iters"]


def test_instance_follows_the_quaternionisation_of_example_4():
    d = qsynth.krylov_instance(3)
    A, As = d["A"], d["As"]
    assert A.shape == (4, 238, 238) and d["B"].shape == (4, 238, 3)
    assert np.array_equal(A[1], -As) and np.array_equal(A[2], 2 * As) and np.array_equal(A[3], 1.5 * As)
    assert not np.allclose(As, As.T)
    assert 0.0 <= d["B"].min() and d["B"].max() < 1.0
