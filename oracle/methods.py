"""The hyperpower-family iterations, step by step in float64 (oracle; test infrastructure only).

Notation follows the paper: A in Q^{m x n}, X_j in Q^{n x m}, R_j = I - A X_j with I = I_m
("right" residual side, exactly as Algorithms 1-3 print it).  The "left" side uses R'_j = I_n - X_j A
and the push-through identity X p(A X) = p(X A) X, valid for every polynomial p; it produces the same
iterates in exact arithmetic and is the form whose residual lives on the smaller side when m > n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .quat import qmul, qH, qeye, fro, sigma_max, modulus

# ----------------------------------------------------------------------------------------------
# coefficients, from their closed forms
# ----------------------------------------------------------------------------------------------
_R93 = math.sqrt(93.0)
_R5 = math.sqrt(5.0)

#: QSAI golden-ratio scalars beta_1, beta_2 (Section 3, QSAI; Algorithm 2 input).
QSAI_BETA = ((1.0 + _R5) / 2.0, (1.0 - _R5) / 2.0)

#: QHPI19 coefficients (Section 3, QHPI19: solution of the coefficient system and the secondary
#: quadratic factorization).
QHPI19 = {
    "a1": 5.0 / 496.0 * (31.0 + _R93),
    "a2": (3.0 + _R93) / 8.0,
    "a3": 0.5,
    "b1": -5.0 / 496.0 * (_R93 - 31.0),
    "b2": (3.0 - _R93) / 8.0,
    "b3": 0.5,
    "c1": 3.0 / 8.0,
    "c2": 321.0 / 1984.0,
    "d1": (math.sqrt(27.0 - 2.0 * _R93) + 1.0) / 4.0,
    "d2": (1.0 - math.sqrt(27.0 - 2.0 * _R93)) / 4.0,
    "d3": (5.0 * _R93 - 93.0) / 496.0,
    "e1": (-93.0 - 5.0 * _R93) / 496.0,
    "e2": -_R93 / 4.0,
}

METHODS = ("ns", "hpi", "qsai", "qhpi19", "qrapid")

#: GEMMs per iteration as each step below performs them (right side / left side).
def gemms_per_iteration(method: str, order: int, side: str) -> int:
    if method == "ns":
        return 2
    if method == "hpi":
        return order
    if method == "qsai":
        return 6
    if method == "qhpi19":
        return 7
    if method == "qrapid":
        return 8 + 2 * order if side == "right" else 6 + 2 * order
    raise ValueError(method)


def fib(k: int) -> int:
    """a_k = (phi^k - (1-phi)^k)/sqrt 5 extended to negative k (a_{-1} = 1, a_{-2} = -1)."""
    a, b = 0, 1  # a_0, a_1
    if k >= 0:
        for _ in range(k):
            a, b = b, a + b
        return a
    # a_{k} = a_{k+2} - a_{k+1}
    for _ in range(-k):
        a, b = b - a, a
    return a


def qrapid_exponents(N: int) -> tuple[int, int]:
    """(a_{N+2}, nu_N) with nu_N = 11 a_{N-1} + 7 a_{N-2} + 1 (Theorem on QRAPID convergence)."""
    return fib(N + 2), 11 * fib(N - 1) + 7 * fib(N - 2) + 1


def scalar_residual_map(method: str, order: int):
    """g with R_{j+1} = g(R_j) (for any X_j, right side): NS rho^2, HPI(p) rho^p, QSAI rho^10,
    QHPI19 rho^19 (convergence theorems of Section 3), QRAPID 4^{-a}(3+rho)^a rho^nu."""
    if method == "ns":
        return lambda r: r ** 2
    if method == "hpi":
        return lambda r: r ** order
    if method == "qsai":
        return lambda r: r ** 10
    if method == "qhpi19":
        return lambda r: r ** 19
    if method == "qrapid":
        a, nu = qrapid_exponents(order)
        return lambda r: (0.25 * (3.0 + r)) ** a * r ** nu
    raise ValueError(method)


def convergence_order(method: str, order: int) -> int:
    if method == "ns":
        return 2
    if method == "hpi":
        return order
    if method == "qsai":
        return 10
    if method == "qhpi19":
        return 19
    return qrapid_exponents(order)[1]


# ----------------------------------------------------------------------------------------------
# one iteration
# ----------------------------------------------------------------------------------------------
def step_ns(A, X, side="right"):
    """Quaternion Newton--Schulz X_{j+1} = X_j (2I - A X_j) (Section 1, QNS)."""
    if side == "right":
        I = qeye(A.shape[1])
        return qmul(X, 2.0 * I - qmul(A, X))
    I = qeye(A.shape[2])
    return qmul(2.0 * I - qmul(X, A), X)


def step_hpi(A, X, p, side="right"):
    """Hyperpower of order p: X_{j+1} = X_j (I + R_j + ... + R_j^{p-1}) (Definition of QHPIM),
    evaluated in Horner form S <- I + R S, p - 1 times from S = I (p GEMMs with the residual and update)."""
    if p < 2:
        raise ValueError("hyperpower order must be >= 2")
    if side == "right":
        I = qeye(A.shape[1])
        R = I - qmul(A, X)
    else:
        I = qeye(A.shape[2])
        R = I - qmul(X, A)
    S = I + R
    for _ in range(p - 2):
        S = I + qmul(R, S)
    return qmul(X, S) if side == "right" else qmul(S, X)


def step_qsai(A, X, side="right"):
    """QSAI (Algorithm 2): R = I - A X; Q = (I + b1 R^2 + R^4)(I + b2 R^2 + R^4); X+ = X (I + R) Q."""
    b1, b2 = QSAI_BETA
    if side == "right":
        I = qeye(A.shape[1])
        R = I - qmul(A, X)
    else:
        I = qeye(A.shape[2])
        R = I - qmul(X, A)
    R2 = qmul(R, R)
    R4 = qmul(R2, R2)
    Q = qmul(I + b1 * R2 + R4, I + b2 * R2 + R4)
    if side == "right":
        return qmul(qmul(X, I + R), Q)
    return qmul(qmul(I + R, Q), X)


def step_qhpi19(A, X, side="right", literal=False):
    """QHPI19 (Algorithm 3): residual powers R, R^2, R^4; U = (I + d1 R^2 + R^4)(I + d2 R^2 + R^4);
    V = U + d3 R^2; W = U + e1 R^2 + e2 R^4; Gamma = V W + c1 R^2 + c2 R^4; X+ = X (I + (R + R^2) Gamma).

    Algorithm 3 also lists R^8 and R^16, which nothing uses; ``literal=True`` forms them anyway (cost only).
    """
    c = QHPI19
    if side == "right":
        I = qeye(A.shape[1])
        R = I - qmul(A, X)
    else:
        I = qeye(A.shape[2])
        R = I - qmul(X, A)
    R2 = qmul(R, R)
    R4 = qmul(R2, R2)
    if literal:
        R8 = qmul(R4, R4)
        qmul(R8, R8)
    U = qmul(I + c["d1"] * R2 + R4, I + c["d2"] * R2 + R4)
    V = U + c["d3"] * R2
    W = U + c["e1"] * R2 + c["e2"] * R4
    G = qmul(V, W) + c["c1"] * R2 + c["c2"] * R4
    T = I + qmul(R + R2, G)
    return qmul(X, T) if side == "right" else qmul(T, X)


def step_qrapid(A, X, N, side="right"):
    """QRAPID (Algorithm 1) with step parameter N >= 0.

    Right side, as printed: P = A X; U = 1/4 X (13I - P(15I - P(7I - P))); V = U + X (I - A U);
    Y_0 = U, W_0 = V, Z_l = W_{l-1} + Y_{l-1}(I - A W_{l-1}), Y_l = W_{l-1}, W_l = Z_l (l = 1..N);
    Z_N = V when N = 0; X+ = Z_N + X (I - A Z_N).
    Left side: every X f(A X) becomes f(X A) X and Y (I - A W) becomes Y - (Y A) W.
    """
    if N < 0:
        raise ValueError("QRAPID step parameter N must be >= 0")
    if side == "right":
        I = qeye(A.shape[1])
        P = qmul(A, X)
        U = 0.25 * qmul(X, 13.0 * I - qmul(P, 15.0 * I - qmul(P, 7.0 * I - P)))
        V = U + qmul(X, I - qmul(A, U))
        Y, W = U, V
        Zc = V
        for _ in range(N):
            Zc = W + qmul(Y, I - qmul(A, W))
            Y, W = W, Zc
        return Zc + qmul(X, I - qmul(A, Zc))
    I = qeye(A.shape[2])
    Q = qmul(X, A)
    U = 0.25 * qmul(13.0 * I - qmul(Q, 15.0 * I - qmul(Q, 7.0 * I - Q)), X)
    V = U + X - qmul(Q, U)
    Y, W = U, V
    Zc = V
    for _ in range(N):
        Zc = W + Y - qmul(qmul(Y, A), W)
        Y, W = W, Zc
    return Zc + X - qmul(Q, Zc)


def step(A, X, method, order=None, side="right"):
    """One iteration of `method` (ns | hpi | qsai | qhpi19 | qrapid) with its order parameter."""
    if method == "ns":
        return step_ns(A, X, side)
    if method == "hpi":
        return step_hpi(A, X, order, side)
    if method == "qsai":
        return step_qsai(A, X, side)
    if method == "qhpi19":
        return step_qhpi19(A, X, side)
    if method == "qrapid":
        return step_qrapid(A, X, 5 if order is None else order, side)
    raise ValueError(f"unknown method {method!r}")


# ----------------------------------------------------------------------------------------------
# scaling (initial iterate X_0 = alpha A^H)
# ----------------------------------------------------------------------------------------------
def alpha_sigma(A) -> float:
    """alpha = 1 / sigma_max(A^C)^2 (scaling step of Algorithms 1-3)."""
    return 1.0 / sigma_max(A) ** 2


def alpha_frobenius(A) -> float:
    """alpha = 1 / ||A||_F^2 (Section 4 experimental setup)."""
    return 1.0 / fro(A) ** 2


_MASK64 = (1 << 64) - 1


def splitmix64(counter: int, seed: int) -> int:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based generator:
    state = seed + (counter + 1) * 0x9E3779B97F4A7C15, then the published finaliser."""
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def power_start_vector(n: int, seed: int) -> np.ndarray:
    """Start vector of the power iteration: (4, n, 1) planes, entry (p, j) = u(splitmix64(p*n + j)),
    u(z) = (z >> 11) * 2^-52 - 1 in [-1, 1)."""
    v = np.empty((4, n, 1))
    for p in range(4):
        for j in range(n):
            z = splitmix64(p * n + j, seed)
            v[p, j, 0] = (z >> 11) * (2.0 ** -52) - 1.0
    return v


def power_sigma1_sq(A, steps: int, seed: int = 0x5EED) -> float:
    """Estimate sigma_1^2 by `steps` power steps on A^H A: v <- v/||v||, w = A v, lambda = ||w||^2,
    v <- A^H w; returns the last lambda (a Rayleigh quotient, hence <= sigma_1^2).

    This replaces the SVD of A^C in the scaling step (the paper leaves that cost uncounted).
    """
    if steps < 1:
        raise ValueError("steps must be >= 1")
    v = power_start_vector(A.shape[2], seed)
    AH = qH(A)
    lam = 0.0
    for _ in range(steps):
        v = v / fro(v)
        w = qmul(A, v)
        lam = fro(w) ** 2
        v = qmul(AH, w)
    return lam


def features(A, steps: int, seed: int = 0x5EED) -> dict:
    """Cheap scaling features: power-iteration sigma_1^2 estimate, ||A||_F, ||A||_1, ||A||_inf, shape."""
    mod = modulus(A)
    return {
        "sigma1_sq": power_sigma1_sq(A, steps, seed),
        "fro": float(np.sqrt(np.sum(mod * mod))),
        "norm1": float(np.max(np.sum(mod, axis=0))),
        "norminf": float(np.max(np.sum(mod, axis=1))),
        "m": A.shape[1],
        "n": A.shape[2],
    }


def x0(A, alpha: float) -> np.ndarray:
    """X_0 = alpha A^H (Theorem 1; the paper's A^T in Section 4 is read as A^H)."""
    return alpha * qH(A)


# ----------------------------------------------------------------------------------------------
# Penrose residuals (Section 4, error metrics)
# ----------------------------------------------------------------------------------------------
def residuals(A, X) -> dict:
    """E1 = ||AXA - A||_F, E2 = ||XAX - X||_F, E3 = ||(AX)^H - AX||_F, E4 = ||(XA)^H - XA||_F, and
    relative forms E1/||A||_F, E2/||X||_F, E3/||AX||_F, E4/||XA||_F."""
    AX = qmul(A, X)
    XA = qmul(X, A)
    E1 = fro(qmul(AX, A) - A)
    E2 = fro(qmul(XA, X) - X)
    E3 = fro(qH(AX) - AX)
    E4 = fro(qH(XA) - XA)
    nA, nX, nAX, nXA = fro(A), fro(X), fro(AX), fro(XA)
    return {
        "E": (E1, E2, E3, E4),
        "E_rel": (E1 / nA, E2 / nX if nX else math.inf, E3 / nAX if nAX else 0.0, E4 / nXA if nXA else 0.0),
    }


def penrose_projection(A, X) -> np.ndarray:
    """(X A)^H X (A X)^H (Section 2): A^dagger is a fixed point, since (b)-(d) give (XA)^H X (AX)^H = XAXAX = X.
    Its rows lie in range(A^H) and its columns in range(A), the invariants every exact iterate keeps
    (Proposition 3.1)."""
    return qmul(qmul(qH(qmul(X, A)), X), qH(qmul(A, X)))


def e1_rel(A, X) -> float:
    return fro(qmul(qmul(A, X), A) - A) / fro(A)


def e2_rel(A, X) -> float:
    return fro(qmul(qmul(X, A), X) - X) / fro(X)


# ----------------------------------------------------------------------------------------------
# full solve with the stop rules
# ----------------------------------------------------------------------------------------------
@dataclass
class Result:
    X: np.ndarray
    iters: int               # updates performed, including the one that triggered the stop
    returned: int            # index j of the returned iterate X_j
    reason: str              # tol | rise | max_iter | diverged
    alpha: float
    dx: list = field(default_factory=list)   # ||X_{j+1} - X_j||_F per update
    xn: list = field(default_factory=list)   # ||X_{j+1}||_F per update


def solve(A, method, order=None, alpha=None, tol=1e-10, max_iter=500, stop="dx_abs",
          side="right", X0=None, keep=False) -> Result:
    """Run `method` from X_0 = alpha A^H (or the given X0) until the stop rule fires.

    stop rules:
      dx_abs  ||X_{j+1} - X_j||_F < tol (Algorithms 1-3, stopping test)
      dx_rel  ||X_{j+1} - X_j||_F <= tol ||X_{j+1}||_F
      e1_rel  ||A X_{j+1} A - A||_F <= tol ||A||_F
      guarded relative change d_j <= tol, or the first rise d_j > d_{j-1} once d has dropped below
              half its running maximum; on a rise the returned iterate is whichever of X_{j*-1},
              X_{j*} (j* = argmin d) has the smaller E2_rel (float64 decision).
    The iteration count is the number of updates performed, including the last.
    Divergence: a non-finite iterate, or ||X||_F ||A||_F above 1e20 (far beyond any pseudoinverse of
    a matrix this code can represent), is reported as reason 'diverged'.
    """
    if alpha is None:
        alpha = alpha_sigma(A)
    X = x0(A, alpha) if X0 is None else X0.copy()
    dx, xn = [], []
    hist = {0: X} if keep else {}
    prev = None       # X_{j-1} kept for the guarded rule
    best = None       # (d, j, X_{j-1}, X_j)
    dmax = 0.0
    nA = fro(A)
    for j in range(1, max_iter + 1):
        Xn = step(A, X, method, order, side)
        if not np.all(np.isfinite(Xn)):
            return Result(X, j, j - 1, "diverged", alpha, dx, xn)
        d_abs = fro(Xn - X)
        nrm = fro(Xn)
        dx.append(d_abs)
        xn.append(nrm)
        if keep:
            hist[j] = Xn
        if nrm * nA > 1e20:
            return Result(Xn, j, j, "diverged", alpha, dx, xn)
        if stop == "dx_abs":
            if d_abs < tol:
                return Result(Xn, j, j, "tol", alpha, dx, xn)
        elif stop == "dx_rel":
            if d_abs <= tol * nrm:
                return Result(Xn, j, j, "tol", alpha, dx, xn)
        elif stop == "e1_rel":
            if e1_rel(A, Xn) <= tol:
                return Result(Xn, j, j, "tol", alpha, dx, xn)
        elif stop == "guarded":
            d = d_abs / nrm
            if d <= tol:
                return Result(Xn, j, j, "tol", alpha, dx, xn)
            dprev = dx[-2] / xn[-2] if len(dx) >= 2 else None
            if best is None or d < best[0]:
                best = (d, j, X, Xn)
            if dprev is not None and d > dprev and dprev < 0.5 * dmax:
                _, js, Xa, Xb = best
                if e2_rel(A, Xa) < e2_rel(A, Xb):
                    return Result(Xa, j, js - 1, "rise", alpha, dx, xn)
                return Result(Xb, j, js, "rise", alpha, dx, xn)
            dmax = max(dmax, d)
        else:
            raise ValueError(f"unknown stop rule {stop!r}")
        prev, X = X, Xn
    return Result(X, max_iter, max_iter, "max_iter", alpha, dx, xn)


def iterate(A, X0, method, order, side, count) -> list:
    """X_0 .. X_count (exactly `count` updates, no stop rule)."""
    out = [X0]
    X = X0
    for _ in range(count):
        X = step(A, X, method, order, side)
        out.append(X)
    return out


# ----------------------------------------------------------------------------------------------
# exact-arithmetic spectral model (Theorem 1 proof: X_0 = alpha A^H keeps every iterate of the form
# V diag(x) U^H, and R_{j+1} = g(R_j) acts on each singular value separately)
# ----------------------------------------------------------------------------------------------
def spectral_rho(s, alpha, method, order, count) -> np.ndarray:
    """rho^{(j)}_i = 1 - s_i x^{(j)}_i for j = 0..count, with rho^{(0)} = 1 - alpha s_i^2."""
    g = scalar_residual_map(method, order)
    rho = 1.0 - alpha * np.asarray(s, dtype=np.float64) ** 2
    out = [rho]
    for _ in range(count):
        rho = g(rho)
        out.append(rho)
    return np.array(out)


def spectral_iterate(U, s, V, alpha, method, order, j) -> np.ndarray:
    """X_j = V diag((1 - rho^{(j)}_i) / s_i) U^H for A = U diag(s) V^H."""
    rho = spectral_rho(s, alpha, method, order, j)[-1]
    x = (1.0 - rho) / s
    return qmul(V * x[None, None, :], qH(U))


def spectral_e1_rel(s, alpha, method, order, count) -> np.ndarray:
    """E1_rel(X_j) = sqrt(sum s_i^2 rho_i^2 / sum s_i^2), j = 0..count."""
    s = np.asarray(s, dtype=np.float64)
    rho = spectral_rho(s, alpha, method, order, count)
    return np.sqrt(np.sum((s * rho) ** 2, axis=1) / np.sum(s * s))


def spectral_dx_iterations(s, alpha, method, order, tol, max_iter=500) -> int:
    """Smallest j >= 1 with ||X_j - X_{j-1}||_F < tol in exact arithmetic (the stopping test of
    Algorithms 1-3), max_iter + 1 if never.  X_j - X_{j-1} = V diag((rho^{(j-1)} - rho^{(j)}) / s) U^H
    and V, U have orthonormal columns, so its Frobenius norm is that of the diagonal."""
    s = np.asarray(s, dtype=np.float64)
    g = scalar_residual_map(method, order)
    rho = 1.0 - alpha * s ** 2
    for j in range(1, max_iter + 1):
        rn = g(rho)
        if not np.all(np.isfinite(rn)) or np.max(np.abs(rn)) > 1e30:
            return max_iter + 1
        if math.sqrt(np.sum(((rho - rn) / s) ** 2)) < tol:
            return j
        rho = rn
    return max_iter + 1


def spectral_iterations(s, alpha, method, order, tol, max_iter=500) -> int:
    """Smallest j >= 1 with E1_rel(X_j) <= tol in exact arithmetic (max_iter + 1 if never)."""
    s = np.asarray(s, dtype=np.float64)
    g = scalar_residual_map(method, order)
    rho = 1.0 - alpha * s ** 2
    den = np.sum(s * s)
    for j in range(1, max_iter + 1):
        rho = g(rho)
        if not np.all(np.isfinite(rho)) or np.max(np.abs(rho)) > 1e30:
            return max_iter + 1
        if math.sqrt(np.sum((s * rho) ** 2) / den) <= tol:
            return j
    return max_iter + 1
