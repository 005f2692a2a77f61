"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: the worked example's printed
numbers, textbook identities of the quaternion algebra, the closed-form Moore--Penrose inverses,
the convergence theorems' residual laws, the coefficient identities, the exact-arithmetic spectral
model, Proposition 3.1 and Theorem 1.
"""
import math

import numpy as np
import pytest

import qsynth
from oracle import quat as Q
from oracle import methods as M

METHOD_CASES = [("ns", None), ("hpi", 3), ("hpi", 7), ("qsai", None), ("qhpi19", None),
                ("qrapid", 0), ("qrapid", 1), ("qrapid", 2), ("qrapid", 3), ("qrapid", 5)]


def rand_q(seed, m, n, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal((4, m, n))


def qpow(R, k):
    n = R.shape[1]
    out = Q.qeye(n)
    for _ in range(k):
        out = Q.qmul(out, R)
    return out


# ------------------------------------------------------------------ Example 1 (Section 4)
def test_example1_alpha(example1):
    A, _, alpha, _ = example1
    assert M.alpha_sigma(A) == pytest.approx(alpha, rel=5e-7)


def test_example1_pinv_svd_matches_printed(example1):
    A, P, _, _ = example1
    X = Q.pinv_svd(A)
    # printed to 4 decimals: half a unit of the last digit, plus float slack
    assert np.max(np.abs(X - P)) <= 5.0e-5 + 1e-9


@pytest.mark.parametrize("method,order", [("qsai", None), ("qhpi19", None), ("qrapid", 1), ("qrapid", 2)])
def test_example1_iterations_and_result(example1, method, order):
    A, P, alpha, iters = example1
    r = M.solve(A, method, order, alpha=M.alpha_sigma(A), tol=1e-10, stop="dx_abs", side="right")
    assert r.reason == "tol"
    assert r.iters == iters[method]
    assert np.max(np.abs(r.X - P)) <= 5.0e-5 + 1e-9
    E = M.residuals(A, r.X)["E"]
    assert max(E) < 1e-13


def test_example1_conjugate_transpose_reading(example1):
    """X_0 = alpha A^T without conjugation does not converge (the paper's A^T is read as A^H)."""
    A, _, _, _ = example1
    alpha = M.alpha_sigma(A)
    XT = alpha * np.stack([A[0].T, A[1].T, A[2].T, A[3].T])
    r = M.solve(A, "qhpi19", alpha=alpha, tol=1e-10, stop="dx_abs", X0=XT, max_iter=30)
    assert r.reason in ("diverged", "max_iter")


def test_example1_rank_two(example1):
    A, _, _, _ = example1
    s = Q.singular_values(A)
    assert s[2] < 1e-12 * s[0]
    X = Q.pinv_svd(A)
    # row 3 = 2 * row 2 of A gives column 3 = 2 * column 2 of the pseudoinverse
    np.testing.assert_allclose(X[:, :, 2], 2.0 * X[:, :, 1], atol=1e-14)


# ------------------------------------------------------------------ quaternion algebra (Section 2)
def _unit(idx):
    e = np.zeros((4, 1, 1))
    e[idx, 0, 0] = 1.0
    return e


def test_hamilton_units():
    one, i, j, k = (_unit(t) for t in range(4))
    for u in (i, j, k):
        np.testing.assert_array_equal(Q.qmul(u, u), -one)
    np.testing.assert_array_equal(Q.qmul(i, j), k)
    np.testing.assert_array_equal(Q.qmul(j, k), i)
    np.testing.assert_array_equal(Q.qmul(k, i), j)
    np.testing.assert_array_equal(Q.qmul(j, i), -k)
    np.testing.assert_array_equal(Q.qmul(Q.qmul(i, j), k), -one)


def test_complex_adjoint_is_homomorphism():
    A, B = rand_q(1, 7, 5), rand_q(2, 5, 6)
    np.testing.assert_allclose(Q.cadj(Q.qmul(A, B)), Q.cadj(A) @ Q.cadj(B), atol=1e-12)
    np.testing.assert_allclose(Q.cadj(Q.qH(A)), Q.cadj(A).conj().T, atol=0)
    np.testing.assert_array_equal(Q.from_cadj(Q.cadj(A)), A)


def test_product_is_associative_and_noncommutative():
    A, B, C = rand_q(3, 4, 4), rand_q(4, 4, 4), rand_q(5, 4, 4)
    np.testing.assert_allclose(Q.qmul(Q.qmul(A, B), C), Q.qmul(A, Q.qmul(B, C)), atol=1e-12)
    assert np.max(np.abs(Q.qmul(A, B) - Q.qmul(B, A))) > 1e-3
    np.testing.assert_allclose(Q.qH(Q.qmul(A, B)), Q.qmul(Q.qH(B), Q.qH(A)), atol=1e-12)


def test_norms():
    p, q = rand_q(6, 1, 1), rand_q(7, 1, 1)
    assert Q.modulus(Q.qmul(p, q))[0, 0] == pytest.approx(Q.modulus(p)[0, 0] * Q.modulus(q)[0, 0], rel=1e-14)
    A = rand_q(8, 9, 6)
    assert np.linalg.norm(Q.cadj(A)) ** 2 == pytest.approx(2 * Q.fro(A) ** 2, rel=1e-13)
    s1 = Q.singular_values(A)[0]
    assert s1 <= math.sqrt(Q.norm1(A) * Q.norminf(A)) * (1 + 1e-12)
    assert s1 <= Q.fro(A)
    # ||A||_1 = ||A^H||_inf
    assert Q.norm1(A) == pytest.approx(Q.norminf(Q.qH(A)), rel=1e-14)


# ------------------------------------------------------------------ definitions of A^dagger
@pytest.mark.parametrize("shape", [(5, 3), (3, 5), (4, 4)])
def test_pinv_svd_satisfies_penrose(shape):
    A = rand_q(10 + shape[0], *shape)
    X = Q.pinv_svd(A)
    E = M.residuals(A, X)["E"]
    assert max(E) < 1e-12


def test_pinv_closed_forms():
    A = rand_q(20, 9, 5)
    np.testing.assert_allclose(Q.pinv_svd(A), Q.pinv_full_column_rank(A), atol=1e-12)
    B = rand_q(21, 5, 9)
    np.testing.assert_allclose(Q.pinv_svd(B), Q.pinv_full_row_rank(B), atol=1e-12)


def test_inverse_square():
    """A^{-1} of a nonsingular square quaternion matrix: both products with A are the identity, it equals the
    SVD pseudoinverse, and on a constructed U diag(s) V^H it is V diag(1/s) U^H."""
    A = rand_q(22, 7, 7)
    X = Q.inverse_square(A)
    np.testing.assert_allclose(Q.qmul(A, X), Q.qeye(7), atol=1e-12)
    np.testing.assert_allclose(Q.qmul(X, A), Q.qeye(7), atol=1e-12)
    np.testing.assert_allclose(X, Q.pinv_svd(A), atol=1e-12)
    inst = qsynth.small_spectral_instance(23, 6, 6, [4.0, 2.0, 1.0, 0.5, 0.25, 0.125])
    np.testing.assert_allclose(Q.inverse_square(inst["A"]), Q.pinv_from_factors(inst["U"], inst["s"], inst["V"]),
                               atol=1e-12)
    # a 1 x 1 quaternion: q^{-1} = conj(q) / |q|^2
    qv = np.array([1.0, 2.0, 2.0, 4.0]).reshape(4, 1, 1)
    np.testing.assert_allclose(Q.inverse_square(qv)[:, 0, 0], np.array([1.0, -2.0, -2.0, -4.0]) / 25.0, rtol=1e-15)
    with pytest.raises(ValueError):
        Q.inverse_square(rand_q(24, 3, 4))


def test_pinv_unitary_is_adjoint():
    U = qsynth.stiefel(30, 8, 8)
    np.testing.assert_allclose(Q.qmul(Q.qH(U), U), Q.qeye(8), atol=1e-12)
    np.testing.assert_allclose(Q.pinv_svd(U), Q.qH(U), atol=1e-12)


def test_pinv_from_factors():
    inst = qsynth.small_spectral_instance(31, 10, 7, [3.0, 1.0, 0.25, 0.1])
    np.testing.assert_allclose(Q.singular_values(inst["A"])[:4], inst["s"], rtol=1e-12)
    np.testing.assert_allclose(Q.pinv_from_factors(inst["U"], inst["s"], inst["V"]), Q.pinv_svd(inst["A"]),
                               atol=1e-12)


# ------------------------------------------------------------------ coefficient identities
def test_qhpi19_coefficients():
    c = M.QHPI19
    P = np.polynomial.polynomial
    q1 = [1.0, c["d1"], 1.0]
    q2 = [1.0, c["d2"], 1.0]
    U = P.polymul(q1, q2)
    G1 = P.polyadd(U, [0.0, c["d3"]])
    G2 = P.polyadd(U, [0.0, c["e1"], c["e2"]])
    # Gamma_1 and Gamma_2 in the variable y = R^2: 1 + a1 y + a2 y^2 + a3 y^3 + y^4
    np.testing.assert_allclose(G1, [1.0, c["a1"], c["a2"], c["a3"], 1.0], atol=1e-14)
    np.testing.assert_allclose(G2, [1.0, c["b1"], c["b2"], c["b3"], 1.0], atol=1e-14)
    Gam = P.polyadd(P.polymul(G1, G2), [0.0, c["c1"], c["c2"]])
    # Gamma = I + R^2 + ... + R^16 is sum_{k=0}^{8} y^k
    np.testing.assert_allclose(Gam, np.ones(9), atol=1e-13)
    # and (x + x^2) Gamma(x^2) + 1 = sum_{k=0}^{18} x^k: the order-19 hyperpower polynomial
    Gx = np.zeros(17)
    Gx[0::2] = Gam
    full = P.polyadd([1.0], P.polymul([0.0, 1.0, 1.0], Gx))
    np.testing.assert_allclose(full, np.ones(19), atol=1e-13)


def test_qsai_coefficients():
    b1, b2 = M.QSAI_BETA
    P = np.polynomial.polynomial
    assert b1 + b2 == pytest.approx(1.0) and b1 * b2 == pytest.approx(-1.0)
    q = P.polymul([1.0, b1, 1.0], [1.0, b2, 1.0])
    np.testing.assert_allclose(q, np.ones(5), atol=1e-14)
    # (1 + x) Q(x^2) = 1 + x + ... + x^9
    Qx = np.zeros(9)
    Qx[0::2] = q
    np.testing.assert_allclose(P.polymul([1.0, 1.0], Qx), np.ones(10), atol=1e-14)


def test_qrapid_exponents():
    # Theorem on QRAPID: orders 5, 8, 12 for N = 0, 1, 2 and nu_5 = 48
    assert [M.qrapid_exponents(N)[1] for N in range(6)] == [5, 8, 12, 19, 30, 48]
    assert [M.fib(k) for k in range(-2, 8)] == [-1, 1, 0, 1, 1, 2, 3, 5, 8, 13]


# ------------------------------------------------------------------ residual laws R_{j+1} = g(R_j)
def _law_poly(method, order, R):
    """g(R) written with matrix powers from the convergence theorems (independent of the step code)."""
    n = R.shape[1]
    I = Q.qeye(n)
    if method == "ns":
        return qpow(R, 2)
    if method == "hpi":
        return qpow(R, order)
    if method == "qsai":
        return qpow(R, 10)
    if method == "qhpi19":
        return qpow(R, 19)
    a, nu = M.qrapid_exponents(order)
    return (0.25 ** a) * Q.qmul(qpow(3.0 * I + R, a), qpow(R, nu))


@pytest.mark.parametrize("method,order", METHOD_CASES)
@pytest.mark.parametrize("side", ["right", "left"])
def test_residual_law_any_iterate(method, order, side):
    m, n = 7, 5
    A = rand_q(40, m, n)
    # a generic X near A^dagger (not of the form V diag U^H), so that ||R|| < 1 and powers stay tame
    X = Q.pinv_svd(A) + rand_q(41, n, m, 0.02 / Q.fro(A))
    Xn = M.step(A, X, method, order, side)
    I = Q.qeye(m)
    R = I - Q.qmul(A, X)
    Rn = I - Q.qmul(A, Xn)
    expect = _law_poly(method, order, R)
    # R has eigenvalue 1 on the complement of range(A) (m > n) and is a contraction elsewhere
    assert Q.singular_values(R)[0] < 1.1
    scale = max(Q.fro(expect), 1e-300)
    assert Q.fro(Rn - expect) <= 1e-11 * max(1.0, scale) + 1e-13


@pytest.mark.parametrize("method,order", METHOD_CASES)
def test_left_right_same_iterates(method, order):
    A = rand_q(50, 9, 6)
    X = M.x0(A, M.alpha_sigma(A))
    for _ in range(2):
        XR = M.step(A, X, method, order, "right")
        XL = M.step(A, X, method, order, "left")
        assert Q.fro(XR - XL) <= 1e-12 * Q.fro(XR)
        X = XR


def test_gemm_counts_match_paper():
    # Section 3: NS 2, QSAI 6, QHPI19 7 multiplications per iteration; hyperpower order p uses p
    assert M.gemms_per_iteration("ns", 2, "right") == 2
    assert M.gemms_per_iteration("qsai", 10, "right") == 6
    assert M.gemms_per_iteration("qhpi19", 19, "right") == 7
    assert M.gemms_per_iteration("hpi", 19, "right") == 19


# ------------------------------------------------------------------ spectral model of every iterate
@pytest.mark.parametrize("method,order", METHOD_CASES)
def test_iterates_follow_spectral_model(method, order):
    s = np.array([2.0, 1.3, 0.7, 0.2, 0.05])
    inst = qsynth.small_spectral_instance(60, 11, 8, s)
    A = inst["A"]
    alpha = 1.0 / s[0] ** 2
    Xs = M.iterate(A, M.x0(A, alpha), method, order, "right", 3)
    for j, X in enumerate(Xs):
        Xe = M.spectral_iterate(inst["U"], s, inst["V"], alpha, method, order, j)
        assert Q.fro(X - Xe) <= 1e-10 * Q.fro(Xe), (method, order, j)
    e1 = M.spectral_e1_rel(s, alpha, method, order, 3)
    for j, X in enumerate(Xs):
        assert M.e1_rel(A, X) == pytest.approx(e1[j], rel=1e-6, abs=1e-13)


def test_spectral_iteration_count_matches_run():
    s = qsynth.geometric(12, 1.0, 1e-2)
    inst = qsynth.small_spectral_instance(61, 20, 15, s)
    for method, order in [("ns", None), ("qsai", None), ("qhpi19", None), ("qrapid", 5)]:
        alpha = 1.0 / s[0] ** 2
        J = M.spectral_iterations(s, alpha, method, order, 1e-10)
        r = M.solve(inst["A"], method, order, alpha=alpha, tol=1e-10, stop="e1_rel", side="right")
        assert r.iters == J, (method, r.iters, J)


def test_spectral_dx_iteration_count_matches_run():
    """The exact-arithmetic count under the paper's absolute stopping test against the step-by-step
    oracle run with that test, several scalings, on a tall (left residual, I_n) and a wide (right
    residual, I_m) matrix of full rank.  (Where the residual keeps the eigenvalue 1 on a null space -- the
    larger side, or any side of a rank-deficient matrix -- the update multiplies rounding there by the
    order p every step, so a tight absolute test may never be met: not a model case.)"""
    s = qsynth.geometric(15, 3.0, 3e-2)
    for (m, n, side) in [(20, 15, "left"), (15, 20, "right")]:
        inst = qsynth.small_spectral_instance(62, m, n, s)
        for method, order in [("ns", None), ("qsai", None), ("qhpi19", None), ("qrapid", 5), ("hpi", 3)]:
            for mu in (1.0, 0.6, 1.7):
                alpha = mu / s[0] ** 2
                J = M.spectral_dx_iterations(s, alpha, method, order, 1e-9)
                r = M.solve(inst["A"], method, order, alpha=alpha, tol=1e-9, stop="dx_abs", side=side)
                assert r.iters == J, (m, n, method, mu, r.iters, J)
                assert r.dx[-1] < 1e-9 <= (r.dx[-2] if len(r.dx) > 1 else np.inf)


# ------------------------------------------------------------------ Proposition 3.1 and Theorem 1
@pytest.mark.parametrize("method,order", [("ns", None), ("qsai", None), ("qhpi19", None), ("qrapid", 2)])
def test_proposition_invariants(method, order):
    # rank-deficient 9 x 7 of rank 4
    inst = qsynth.small_spectral_instance(70, 9, 7, [1.5, 1.0, 0.4, 0.1])
    A = inst["A"]
    Ad = Q.pinv_from_factors(inst["U"], inst["s"], inst["V"])
    X = M.x0(A, M.alpha_sigma(A))
    for _ in range(3):
        X = M.step(A, X, method, order, "right")
        AX, XA = Q.qmul(A, X), Q.qmul(X, A)
        tol = 1e-12 * max(1.0, Q.fro(X))
        assert Q.fro(Q.qmul(Q.qmul(Ad, A), X) - X) <= tol
        assert Q.fro(Q.qmul(X, Q.qmul(A, Ad)) - X) <= tol
        assert Q.fro(Q.qH(AX) - AX) <= 1e-12 * max(1.0, Q.fro(AX))
        assert Q.fro(Q.qH(XA) - XA) <= 1e-12 * max(1.0, Q.fro(XA))


def test_theorem1_interval():
    A = rand_q(80, 12, 9)
    s1 = Q.singular_values(A)[0]
    ok = M.solve(A, "qhpi19", alpha=1.98 / s1 ** 2, tol=1e-12, stop="e1_rel", max_iter=60)
    assert ok.reason == "tol"
    bad = M.solve(A, "qhpi19", alpha=2.02 / s1 ** 2, tol=1e-12, stop="e1_rel", max_iter=60)
    assert bad.reason == "diverged"
    # rho(R_0) = max |1 - alpha s_i^2| < 1 exactly inside the interval
    s = Q.singular_values(A)
    assert np.max(np.abs(1 - (1.98 / s1 ** 2) * s ** 2)) < 1
    assert np.max(np.abs(1 - (2.02 / s1 ** 2) * s ** 2)) > 1


# ------------------------------------------------------------------ closed forms at the small workload
def test_small_workload_closed_form():
    A = qsynth.c1_instance(0)
    Xc = Q.pinv_full_column_rank(A)
    for method, order in [("ns", None), ("qsai", None), ("qhpi19", None), ("qrapid", 5)]:
        r = M.solve(A, method, order, alpha=M.alpha_sigma(A), tol=1e-12, stop="e1_rel", side="right")
        assert r.reason == "tol"
        assert Q.fro(r.X - Xc) <= 1e-10 * Q.fro(Xc)
        rl = M.solve(A, method, order, alpha=M.alpha_sigma(A), tol=1e-12, stop="e1_rel", side="left")
        assert rl.iters == r.iters


# ------------------------------------------------------------------ scaling helpers
def test_splitmix64_published_vectors():
    # first outputs of SplitMix64 seeded with 0 (reference implementation by S. Vigna)
    assert M.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert M.splitmix64(1, 0) == 0x6E789E6AA1B965F4
    assert M.splitmix64(2, 0) == 0x06C45D188009454F


def test_power_iteration_lower_bound_and_convergence():
    A = rand_q(90, 30, 20)
    s1sq = Q.singular_values(A)[0] ** 2
    prev = 0.0
    for k in (1, 2, 4, 8, 32, 200):
        lam = M.power_sigma1_sq(A, k)
        assert lam <= s1sq * (1 + 1e-12)
        assert lam >= prev * (1 - 1e-12)
        prev = lam
    assert prev == pytest.approx(s1sq, rel=1e-6)


def test_features_definitions():
    A = rand_q(91, 6, 4)
    f = M.features(A, 3)
    assert f["fro"] == pytest.approx(Q.fro(A))
    assert f["norm1"] == pytest.approx(Q.norm1(A))
    assert f["norminf"] == pytest.approx(Q.norminf(A))
    assert (f["m"], f["n"]) == (6, 4)


def test_guarded_stop_fp64_converges_by_tolerance():
    A = qsynth.c1_instance(1)
    r = M.solve(A, "qhpi19", alpha=M.alpha_sigma(A), tol=1e-12, stop="guarded", side="left")
    assert r.reason in ("tol", "rise")
    assert Q.fro(r.X - Q.pinv_full_column_rank(A)) <= 1e-10 * Q.fro(r.X)


# ------------------------------------------------------------------ norms, alpha_F and E1-E4 at hand-computed values
def _qrow(entries):
    """1 x n quaternion row vector from (s, x, y, z) tuples."""
    return np.array(entries, dtype=float).T.reshape(4, 1, len(entries))


def test_norm1_norminf_on_row_and_column_vectors():
    """Section 2's induced norms on a vector: for a 1 x n row the column sums are the entry moduli, so
    ||a||_1 = max_j |a_j| and ||a||_inf = sum_j |a_j|; transposed for an n x 1 column.  Entries chosen with
    integer moduli: |1+2i+2j+4k| = 5, |2+3i+6j| = 7, |1+4i+8j| = 9."""
    a = _qrow([(1, 2, 2, 4), (2, 3, 6, 0), (1, 4, 8, 0)])
    assert Q.norm1(a) == pytest.approx(9.0, rel=1e-15)
    assert Q.norminf(a) == pytest.approx(21.0, rel=1e-15)
    col = np.ascontiguousarray(np.transpose(a, (0, 2, 1)))
    assert Q.norm1(col) == pytest.approx(21.0, rel=1e-15)
    assert Q.norminf(col) == pytest.approx(9.0, rel=1e-15)


def test_norms_of_example1(example1):
    """Example 1's matrix: row 2 is twice row 1, entry moduli squared are 74, 39, 114 / 7, 20, 34 /
    28, 80, 136 (summed by hand from the printed entries), so the largest column sum is sqrt(114) + 3 sqrt(34)
    (column 3) and the largest row sum 2 (sqrt(7) + sqrt(20) + sqrt(34)) (row 3)."""
    A, _, _, _ = example1
    assert Q.norm1(A) == pytest.approx(math.sqrt(114) + 3 * math.sqrt(34), rel=1e-14)
    assert Q.norminf(A) == pytest.approx(2 * (math.sqrt(7) + math.sqrt(20) + math.sqrt(34)), rel=1e-14)
    assert Q.fro(A) ** 2 == pytest.approx(532.0, rel=1e-15)


def test_alpha_frobenius_example1(example1):
    """Section 4's scaling 1/||A||_F^2 on Example 1: the squared components sum to 227 + 61 + 244 = 532
    by rows (by hand), and ||A||_F^2 is also the sum of the squared singular values."""
    A, _, _, _ = example1
    assert M.alpha_frobenius(A) == pytest.approx(1.0 / 532.0, rel=1e-15)
    assert M.alpha_frobenius(A) == pytest.approx(1.0 / float(np.sum(Q.singular_values(A) ** 2)), rel=1e-12)
    # the two scalings differ on this rank-2 matrix (sigma_1^2 < ||A||_F^2)
    assert M.alpha_frobenius(A) < M.alpha_sigma(A)


def test_residuals_at_zero_iterate():
    """X = 0: A X A - A = -A, X A X - X = 0 and A X, X A are zero (Hermitian)."""
    A = rand_q(100, 5, 3)
    r = M.residuals(A, np.zeros((4, 3, 5)))
    E1, E2, E3, E4 = r["E"]
    assert E1 == pytest.approx(Q.fro(A), rel=1e-15)
    assert (E2, E3, E4) == (0.0, 0.0, 0.0)
    assert r["E_rel"][0] == pytest.approx(1.0, rel=1e-15)


def test_residuals_hand_computed_real_case():
    """A = diag(1, 2), X = e_1 e_2^T (real): AX = [[0,1],[0,0]], XA = [[0,2],[0,0]], AXA = [[0,2],[0,0]],
    XAX = 0, so E1 = ||[[-1,2],[0,-2]]|| = 3, E2 = ||X|| = 1, E3 = sqrt 2, E4 = 2 sqrt 2; relative forms
    divide by ||A|| = sqrt 5, ||X|| = 1, ||AX|| = 1 and ||XA|| = 2.  E3 != E4 separates the two Hermitian
    residuals."""
    A = np.zeros((4, 2, 2))
    A[0] = np.diag([1.0, 2.0])
    X = np.zeros((4, 2, 2))
    X[0, 0, 1] = 1.0
    r = M.residuals(A, X)
    np.testing.assert_allclose(r["E"], [3.0, 1.0, math.sqrt(2), 2 * math.sqrt(2)], rtol=1e-15)
    np.testing.assert_allclose(r["E_rel"], [3.0 / math.sqrt(5), 1.0, math.sqrt(2), math.sqrt(2)], rtol=1e-15)


def test_residuals_identity_operator():
    """A = I_2 and the quaternion X = B = [[1+i, 2j], [3, k]] (by hand, with ij = k, jk = i):
    B^H - B = [[-2i, 3-2j], [-3-2j, -2k]] so E3 = E4 = sqrt 34; B - I = [[i, 2j], [3, -1+k]] so E1 = 4;
    B^2 = [[2i+6j, 2i+2j+2k], [3+3i+3k, -1+6j]], B^2 - B = [[-1+i+6j, 2i+2k], [3i+3k, -1+6j-k]] so
    E2 = sqrt 102."""
    B = np.zeros((4, 2, 2))
    B[:, 0, 0] = (1, 1, 0, 0)
    B[:, 0, 1] = (0, 0, 2, 0)
    B[:, 1, 0] = (3, 0, 0, 0)
    B[:, 1, 1] = (0, 0, 0, 1)
    r = M.residuals(Q.qeye(2), B)
    np.testing.assert_allclose(r["E"], [4.0, math.sqrt(102), math.sqrt(34), math.sqrt(34)], rtol=1e-15)


def test_residuals_spectral_iterate():
    """A = U diag(s) V^H (5 x 4, rank 3) and X = V diag(x) U^H with x not 1/s: AXA = U diag(s^2 x) V^H and
    XAX = V diag(x^2 s) U^H, so E1 = ||s^2 x - s||_2, E2 = ||x^2 s - x||_2, and AX = U diag(sx) U^H,
    XA = V diag(sx) V^H are Hermitian (E3 = E4 = 0)."""
    s = np.array([2.0, 1.0, 0.5])
    x = np.array([0.3, 0.8, 1.5])
    inst = qsynth.small_spectral_instance(101, 5, 4, s)
    X = Q.pinv_from_factors(inst["U"], 1.0 / x, inst["V"])   # V diag(x) U^H
    r = M.residuals(inst["A"], X)
    E1, E2, E3, E4 = r["E"]
    assert E1 == pytest.approx(float(np.linalg.norm(s * s * x - s)), rel=1e-12)
    assert E2 == pytest.approx(float(np.linalg.norm(x * x * s - x)), rel=1e-12)
    assert E3 <= 1e-14 and E4 <= 1e-14
    nr = r["E_rel"]
    assert nr[0] == pytest.approx(E1 / float(np.linalg.norm(s)), rel=1e-12)
    assert nr[1] == pytest.approx(E2 / float(np.linalg.norm(x)), rel=1e-12)


def test_penrose_projection():
    """(X A)^H X (A X)^H: A^dagger is a fixed point; on X = A^dagger + E with E supported on the blocks outside
    range(A^H) x range(A) (rows in the null space of A, or columns in the null space of A^H), it returns A^dagger
    up to second order in E, while X A X keeps the mixed blocks (every {2}-inverse is its fixed point)."""
    inst = qsynth.small_spectral_instance(102, 9, 7, [2.0, 1.0, 0.5, 0.25])   # rank 4
    A, U, s, V = inst["A"], inst["U"], inst["s"], inst["V"]
    Ad = Q.pinv_from_factors(U, s, V)
    np.testing.assert_allclose(M.penrose_projection(A, Ad), Ad, atol=1e-12)
    # null-space bases: complements of V (7 x 4 -> 3 more columns) and U (9 x 4 -> 5 more)
    full_V = qsynth.stiefel(103, 7, 7)
    PV = Q.qmul(V, Q.qH(V))
    Vn = full_V - Q.qmul(PV, full_V)                       # columns in null(A)
    PU = Q.qmul(U, Q.qH(U))
    full_U = qsynth.stiefel(104, 9, 9)
    Un = full_U - Q.qmul(PU, full_U)                       # columns in null(A^H)
    eps = 1e-6
    E_nr = eps * Q.qmul(Q.qmul(Vn, rand_q(105, 7, 4)), Q.qH(U))      # rows outside range(A^H), columns in range(A)
    E_rn = eps * Q.qmul(Q.qmul(V, rand_q(106, 4, 9)), Q.qH(Un))      # rows in range(A^H), columns outside range(A)
    X = Ad + E_nr + E_rn
    P = M.penrose_projection(A, X)
    assert Q.fro(P - Ad) <= 1e3 * eps ** 2 * Q.fro(Ad)
    XAX = Q.qmul(Q.qmul(X, A), X)
    assert Q.fro(XAX - Ad) >= 0.5 * Q.fro(E_nr + E_rn)
    # the projection of anything has rows in range(A^H) and columns in range(A)
    Y = rand_q(107, 7, 9)
    PY = M.penrose_projection(A, Y)
    np.testing.assert_allclose(Q.qmul(PV, PY), PY, atol=1e-10 * Q.fro(PY))
    np.testing.assert_allclose(Q.qmul(PY, PU), PY, atol=1e-10 * Q.fro(PY))
