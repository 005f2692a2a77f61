"""Global quaternion Krylov solvers for A X = B (oracle; test infrastructure only).

Section 3.5 and Section 4, Example 4 use the global quaternion FOM and GMRES of the cited reference,
optionally on the left-preconditioned system M A X = M B with a QSAI approximate inverse M.  Restated
here from the textbook global Arnoldi process: the basis V_1, V_2, ... of n x m quaternion matrices is
orthonormal in <X, Y> = Re tr(X^H Y) (modified Gram-Schmidt), with A V_j = sum_i h_ij V_i; GMRES takes
y minimising ||beta e_1 - Hbar_k y||_2, FOM solves H_k y = beta e_1, and X_k = X_0 + sum_i y_i V_i.
The residual norms come from Givens rotations of Hbar_k (FOM's is GMRES's divided by the last cosine).
"""
from __future__ import annotations

import numpy as np

from . import quat as Q


def inner(X: np.ndarray, Y: np.ndarray) -> float:
    """<X, Y> = Re tr(X^H Y): the sum over planes of the elementwise products."""
    return float(np.sum(X * Y))


def operator(A, M=None):
    """V -> A V, or M (A V) for the left-preconditioned system."""
    if M is None:
        return lambda V: Q.qmul(A, V)
    return lambda V: Q.qmul(M, Q.qmul(A, V))


def solve(A: np.ndarray, B: np.ndarray, method: str = "gmres", M: np.ndarray | None = None,
          X0: np.ndarray | None = None, tol: float = 1e-6, max_iter: int = 3000) -> dict:
    """Gl-QGMRES / Gl-QFOM without restart.  Stops when RR = ||B - A X_k|| / ||B - A X_0|| <= tol (Example
    4).  The method tracks the iterated system's relative residual ||M (B - A X_k)|| / ||M (B - A X_0)||
    (history, rr); with M, RR is evaluated at every step once that tracked value is <= tol.  Returns X,
    iters, rr, true_rr, history, and the basis and Hessenberg (for checks)."""
    op = operator(A, M)
    X0 = np.zeros((4, A.shape[2], B.shape[2])) if X0 is None else X0
    R0 = B - Q.qmul(A, X0)
    Z0 = R0 if M is None else Q.qmul(M, R0)
    beta = np.sqrt(inner(Z0, Z0))
    V = [Z0 / beta]
    H = np.zeros((max_iter + 1, max_iter))
    cs, sn = [], []
    g = [beta]
    hist = []
    k = 0
    for j in range(max_iter):
        W = op(V[j])
        for i in range(j + 1):  # modified Gram-Schmidt
            H[i, j] = inner(V[i], W)
            W = W - H[i, j] * V[i]
        H[j + 1, j] = np.sqrt(inner(W, W))
        col = H[: j + 2, j].copy()
        for i in range(j):
            col[i], col[i + 1] = cs[i] * col[i] + sn[i] * col[i + 1], -sn[i] * col[i] + cs[i] * col[i + 1]
        rho = np.hypot(col[j], col[j + 1])
        c, s = (col[j] / rho, col[j + 1] / rho) if rho > 0 else (1.0, 0.0)
        cs.append(c)
        sn.append(s)
        g.append(-s * g[j])
        g[j] = c * g[j]
        k = j + 1
        res = abs(g[j + 1]) if method == "gmres" else abs(g[j + 1]) / abs(c)
        hist.append(res / beta)
        stop = H[j + 1, j] == 0.0
        if res / beta <= tol:
            # Example 4 stops on the residual of the original system; with M it is checked from here on
            stop = stop or M is None or true_residual(A, B, R0, solution(X0, V, H, k, beta, method)) <= tol
        if stop:
            break
        V.append(W / H[j + 1, j])
    Hk = H[: k + 1, :k]
    y = coefficients(H, k, beta, method)
    X = solution(X0, V, H, k, beta, method)
    true_rr = true_residual(A, B, R0, X)
    return {"X": X, "iters": k, "rr": hist[-1], "true_rr": float(true_rr), "history": hist, "V": V[:k + 1],
            "H": Hk, "beta": beta, "y": y, "converged": true_rr <= tol}


def coefficients(H: np.ndarray, k: int, beta: float, method: str) -> np.ndarray:
    """GMRES: argmin ||beta e_1 - Hbar_k y||_2 (least squares); FOM: H_k y = beta e_1."""
    if method == "gmres":
        return np.linalg.lstsq(H[: k + 1, :k], beta * np.eye(k + 1)[:, 0], rcond=None)[0]
    return np.linalg.solve(H[:k, :k], beta * np.eye(k)[:, 0])


def solution(X0, V, H, k, beta, method):
    y = coefficients(H, k, beta, method)
    return X0 + sum(y[i] * V[i] for i in range(k))


def true_residual(A, B, R0, X) -> float:
    """RR = ||B - A X||_F / ||B - A X_0||_F (Example 4)."""
    R = B - Q.qmul(A, X)
    return float(np.sqrt(inner(R, R) / inner(R0, R0)))
