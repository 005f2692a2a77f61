"""A host evaluation of the methods' update chains in which every product and every stored intermediate is
rounded to FP32 (u = 2^-24), left residual side, NumPy float32 throughout.

Test infrastructure for FP32 tolerances, not an oracle: its outputs are never expected values.  The GPU's FP32
path and this evaluation make the same kinds of rounding errors (one rounding per stored value, dot products
accumulated in FP32) in different orders, so the error of each against the FP64 oracle has the same size in
expectation; a parity bound for the GPU is a small multiple of this evaluation's error.  It follows the
update formulas of Section 3 (Newton-Schulz, QSAI of Algorithm 2, QHPI19 of Algorithm 3, QRAPID of
Algorithm 1) and imports nothing from the oracle or the GPU package.
"""
from __future__ import annotations

import math

import numpy as np

F = np.float32


def qmul(A, B):
    """Hamilton product of FP32 plane stacks, each plane product an FP32 matrix product."""
    a0, a1, a2, a3 = A
    b0, b1, b2, b3 = B
    return np.stack([a0 @ b0 - a1 @ b1 - a2 @ b2 - a3 @ b3,
                     a0 @ b1 + a1 @ b0 + a2 @ b3 - a3 @ b2,
                     a0 @ b2 - a1 @ b3 + a2 @ b0 + a3 @ b1,
                     a0 @ b3 + a1 @ b2 - a2 @ b1 + a3 @ b0]).astype(F)


def eye(n):
    out = np.zeros((4, n, n), dtype=F)
    out[0] = np.eye(n, dtype=F)
    return out


_S93 = math.sqrt(93.0)
_RT = math.sqrt(27.0 - 2.0 * _S93)
_D1, _D2 = F(0.25 * (1.0 + _RT)), F(0.25 * (1.0 - _RT))
_D3, _E1, _E2 = F((5.0 * _S93 - 93.0) / 496.0), F((-93.0 - 5.0 * _S93) / 496.0), F(-0.25 * _S93)
_C1, _C2 = F(3.0 / 8.0), F(321.0 / 1984.0)
_B1, _B2 = F(0.5 * (1.0 + math.sqrt(5.0))), F(0.5 * (1.0 - math.sqrt(5.0)))


def step(A, X, method, order=None):
    """One left-side update X+ = p(I - X A) X in FP32 (A: m x n, X: n x m, both float32)."""
    n = A.shape[2]
    I = eye(n)
    R = (I - qmul(X, A)).astype(F)
    if method == "ns":
        return qmul((I + R).astype(F), X)
    R2 = qmul(R, R)
    R4 = qmul(R2, R2)
    if method == "qsai":
        Q = qmul((I + _B1 * R2 + R4).astype(F), (I + _B2 * R2 + R4).astype(F))
        return qmul(qmul((I + R).astype(F), Q), X)
    if method == "qhpi19":
        U = qmul((I + _D1 * R2 + R4).astype(F), (I + _D2 * R2 + R4).astype(F))
        V = (U + _D3 * R2).astype(F)
        W = (U + _E1 * R2 + _E2 * R4).astype(F)
        G = (qmul(V, W) + _C1 * R2 + _C2 * R4).astype(F)
        T = (I + qmul((R + R2).astype(F), G)).astype(F)
        return qmul(T, X)
    if method == "qrapid":
        N = 5 if order is None else order
        Qm = (I - R).astype(F)  # X A
        U = (F(0.25) * qmul((13 * I - qmul(Qm, (15 * I - qmul(Qm, (7 * I - Qm).astype(F))).astype(F))).astype(F),
                           X)).astype(F)
        V = (U + X - qmul(Qm, U)).astype(F)
        Y, Wm, Z = U, V, V
        for _ in range(N):
            Z = (Wm + Y - qmul(qmul(Y, A), Wm)).astype(F)
            Y, Wm = Wm, Z
        return (Z + X - qmul(Qm, Z)).astype(F)
    raise ValueError(method)


def iterate(A, X0, method, count, order=None):
    """X_count from X_0 in FP32 (inputs rounded to FP32 first)."""
    A = np.asarray(A, dtype=F)
    X = np.asarray(X0, dtype=F)
    for _ in range(count):
        X = step(A, X, method, order)
    return X.astype(np.float64)
