"""CUR approximation and impute-reconstruct completion of Section 5.1 (oracle; test infrastructure only).

With C = A(:, J) and R = A(I, :), the coupling that minimises ||A - C U R||_F is U = C^dagger A R^dagger;
the cross form uses U = W^dagger with W = A(I, J).  Completion alternates a CUR reconstruction X_t of
the filled matrix with re-imposing the observed entries: C_{t+1} = Omega (.) M + (1 - Omega) (.) X_t.
"""
from __future__ import annotations

import numpy as np

from . import quat as Q


def factors(A: np.ndarray, rows, cols):
    """C = A(:, cols), R = A(rows, :), W = A(rows, cols)."""
    rows, cols = np.asarray(rows), np.asarray(cols)
    return A[:, :, cols], A[:, rows, :], A[:, rows][:, :, cols]


def reconstruct(A: np.ndarray, rows, cols) -> tuple[np.ndarray, np.ndarray]:
    """(C U R, U) with U = C^dagger A R^dagger (Section 5.1, the Frobenius-optimal coupling)."""
    C, R, _ = factors(A, rows, cols)
    U = Q.qmul(Q.qmul(Q.pinv_svd(C), A), Q.pinv_svd(R))
    return Q.qmul(Q.qmul(C, U), R), U


def reconstruct_cross(A: np.ndarray, rows, cols) -> np.ndarray:
    """C W^dagger R (Section 5.1, the cross approximation)."""
    C, R, W = factors(A, rows, cols)
    return Q.qmul(Q.qmul(C, Q.pinv_svd(W)), R)


def merge(M: np.ndarray, mask: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Omega (.) M + (1 - Omega) (.) X for every plane (mask nonzero = observed)."""
    return np.where(np.asarray(mask, dtype=bool)[None], M, X)


def complete(M: np.ndarray, mask: np.ndarray, rows, cols, iters: int) -> list:
    """X_0 .. X_{iters-1} of the impute-reconstruct loop from C_0 = Omega (.) M."""
    Ct = merge(M, mask, np.zeros_like(M))
    out = []
    for _ in range(iters):
        X, _ = reconstruct(Ct, rows, cols)
        out.append(X)
        Ct = merge(M, mask, X)
    return out


def psnr(X: np.ndarray, ref: np.ndarray, peak: float = 1.0) -> float:
    """PSNR in dB over the three imaginary (colour) planes."""
    mse = float(np.mean((np.asarray(X)[1:] - np.asarray(ref)[1:]) ** 2))
    return 10.0 * np.log10(peak * peak / mse)
