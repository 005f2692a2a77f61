"""Quaternion matrix algebra in float64 (oracle; test infrastructure only).

A quaternion matrix A = A^(s) + A^(x) i + A^(y) j + A^(z) k in Q^{m x n} is stored as a float64
array of shape (4, m, n) holding the four real component planes (Section 2).
"""
from __future__ import annotations

import numpy as np

S, X, Y, Z = 0, 1, 2, 3


def qmul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A B for quaternion matrices, Hamilton product with i^2 = j^2 = k^2 = ijk = -1 (Section 2).

    Entrywise (a_s + a_x i + a_y j + a_z k)(b_s + b_x i + b_y j + b_z k) expands, using ij = k,
    jk = i, ki = j and the anticommuting reverses, into 16 real products; each term below is one
    float64 matrix product of two planes.
    """
    As, Ax, Ay, Az = A
    Bs, Bx, By, Bz = B
    Cs = As @ Bs - Ax @ Bx - Ay @ By - Az @ Bz
    Cx = As @ Bx + Ax @ Bs + Ay @ Bz - Az @ By
    Cy = As @ By - Ax @ Bz + Ay @ Bs + Az @ Bx
    Cz = As @ Bz + Ax @ By - Ay @ Bx + Az @ Bs
    return np.stack([Cs, Cx, Cy, Cz])


def qH(A: np.ndarray) -> np.ndarray:
    """Conjugate transpose A^H (Section 2): transpose every plane, negate the three imaginary planes."""
    return np.stack([A[0].T, -A[1].T, -A[2].T, -A[3].T])


def qeye(n: int) -> np.ndarray:
    """Quaternion identity I_n: ones on the diagonal of the real plane."""
    I = np.zeros((4, n, n))
    I[0] = np.eye(n)
    return I


def qzeros(m: int, n: int) -> np.ndarray:
    return np.zeros((4, m, n))


def fro(A: np.ndarray) -> float:
    """Frobenius norm: sqrt of the sum of squared moduli = sqrt of the sum of all squared components."""
    return float(np.sqrt(np.sum(A * A)))


def modulus(A: np.ndarray) -> np.ndarray:
    """Entrywise quaternion modulus |a| = sqrt(a_s^2 + a_x^2 + a_y^2 + a_z^2)."""
    return np.sqrt(np.sum(A * A, axis=0))


def norm1(A: np.ndarray) -> float:
    """||A||_1 = max over columns of the sum of entry moduli."""
    return float(np.max(np.sum(modulus(A), axis=0)))


def norminf(A: np.ndarray) -> float:
    """||A||_inf = max over rows of the sum of entry moduli."""
    return float(np.max(np.sum(modulus(A), axis=1)))


def cadj(A: np.ndarray) -> np.ndarray:
    """Complex representation A^C in C^{2m x 2n} (Section 2):
    [[A_s + A_x i,  A_y + A_z i], [-A_y + A_z i,  A_s - A_x i]]."""
    top = np.concatenate([A[0] + 1j * A[1], A[2] + 1j * A[3]], axis=1)
    bot = np.concatenate([-A[2] + 1j * A[3], A[0] - 1j * A[1]], axis=1)
    return np.concatenate([top, bot], axis=0)


def from_cadj(C: np.ndarray) -> np.ndarray:
    """Inverse of ``cadj`` on its image: read the planes back from the top block row."""
    m, n = C.shape[0] // 2, C.shape[1] // 2
    a1, a2 = C[:m, :n], C[:m, n:]
    return np.stack([a1.real, a1.imag, a2.real, a2.imag])


def singular_values(A: np.ndarray) -> np.ndarray:
    """Singular values of A, descending: those of A^C, each of which appears twice (QSVD, Section 2)."""
    sv = np.linalg.svd(cadj(A), compute_uv=False)
    return sv[0::2][: min(A.shape[1], A.shape[2])]


def sigma_max(A: np.ndarray) -> float:
    """sigma_max(A^C) as used by the scaling step of Algorithms 1-3."""
    return float(np.linalg.svd(cadj(A), compute_uv=False)[0])


def pinv_svd(A: np.ndarray, rcond: float | None = None) -> np.ndarray:
    """A^dagger = V Sigma^dagger U^H (Section 2) via the SVD of the complex adjoint.

    Singular values <= rcond * sigma_1 are treated as zero; default rcond = max(m, n) * 2^-52.
    """
    m, n = A.shape[1], A.shape[2]
    if rcond is None:
        rcond = max(m, n) * np.finfo(np.float64).eps
    W, sv, Zh = np.linalg.svd(cadj(A), full_matrices=False)
    keep = sv > rcond * sv[0]
    inv = np.zeros_like(sv)
    inv[keep] = 1.0 / sv[keep]
    P = (Zh.conj().T * inv) @ W.conj().T
    return from_cadj(P)


def pinv_full_column_rank(A: np.ndarray) -> np.ndarray:
    """(A^H A)^{-1} A^H for full column rank A, solved in the complex representation (no explicit inverse)."""
    C = cadj(A)
    G = C.conj().T @ C
    return from_cadj(np.linalg.solve(G, C.conj().T))


def pinv_full_row_rank(A: np.ndarray) -> np.ndarray:
    """A^H (A A^H)^{-1} for full row rank A."""
    C = cadj(A)
    G = C @ C.conj().T
    return from_cadj(np.linalg.solve(G, C).conj().T)


def inverse_square(A: np.ndarray) -> np.ndarray:
    """A^{-1} for a nonsingular square A, which is then its Moore-Penrose inverse (Section 2): the complex adjoint
    of the inverse is the inverse of the complex adjoint (a homomorphism), solved from A^C Z = I by LU.  Its
    relative error is about kappa(A) u, against kappa(A)^2 u for the normal equations of the full-rank form."""
    if A.shape[1] != A.shape[2]:
        raise ValueError("inverse_square: A must be square")
    C = cadj(A)
    return from_cadj(np.linalg.solve(C, np.eye(C.shape[0], dtype=C.dtype)))


def pinv_from_factors(U: np.ndarray, s: np.ndarray, V: np.ndarray) -> np.ndarray:
    """For A = U diag(s) V^H with orthonormal U, V and s > 0: A^dagger = V diag(1/s) U^H (Section 2)."""
    Vs = V / s[None, None, :]
    return qmul(Vs, qH(U))
