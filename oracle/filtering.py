"""Quaternion filter design of Section 5.2 (oracle; test infrastructure only).

The filtered output approximates the clean signal by a quaternion convolution whose coefficients
solve the Toeplitz system X h = s in the least-squares sense: h = X^dagger s (the pseudoinverse of
the data matrix applied to the target), s_hat = X h, and the recovery error is
eps = ||s_hat - s|| / ||s|| (Frobenius norms of the quaternion vectors).
"""
from __future__ import annotations

import numpy as np

from . import quat as Q


def design(X: np.ndarray, s: np.ndarray, Xp: np.ndarray | None = None) -> dict:
    """h = X^dagger s, s_hat = X h and eps (Section 5.2).  X^dagger is the SVD definition
    (quat.pinv_svd) unless a pseudoinverse Xp is passed in."""
    if Xp is None:
        Xp = Q.pinv_svd(X)
    h = Q.qmul(Xp, s)
    s_hat = Q.qmul(X, h)
    return {"h": h, "s_hat": s_hat, "eps": recovery_error(s_hat, s)}


def design_invertible(X: np.ndarray, s: np.ndarray) -> dict:
    """The same quantities for a square invertible X, where X^dagger = X^{-1}: h from a linear solve of
    the complex adjoint system (an O(n^3) route for sizes where the SVD is slow)."""
    h = Q.from_cadj(np.linalg.solve(Q.cadj(X), Q.cadj(s)))
    s_hat = Q.qmul(X, h)
    return {"h": h, "s_hat": s_hat, "eps": recovery_error(s_hat, s)}


def recovery_error(s_hat: np.ndarray, s: np.ndarray) -> float:
    """eps = ||s_hat - s|| / ||s|| (Section 5.2)."""
    return Q.fro(np.asarray(s_hat) - np.asarray(s)) / Q.fro(s)


def toeplitz_columns(X: np.ndarray) -> bool:
    """True when X[i, j] depends only on i - j (the filter-design data matrix is Toeplitz)."""
    return bool(np.array_equal(X[:, 1:, 1:], X[:, :-1, :-1]))
