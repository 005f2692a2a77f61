"""Seeded synthetic quaternion inputs, shared by the GPU path's tests/benchmarks and the CPU oracle.

This module only *builds inputs*: Gaussian component planes, prescribed singular-value spectra and
orthonormal quaternion factors, and the product A = U diag(s) V^H that places a spectrum on them.
It holds none of the pseudoinverse method's arithmetic (no residuals, no hyperpower polynomials,
no scaling rule) and imports neither the oracle nor the GPU package.

Storage convention (both sides): a quaternion matrix A = A_s + A_x i + A_y j + A_z k of shape m x n is
a float64 array of shape (4, m, n), planes in the order (s, x, y, z).

Construction of orthonormal quaternion factors.  The paper's experiments use unseeded Gaussian
matrices (Section 4).  For matrices with a prescribed spectrum we need quaternion matrices with
orthonormal columns.  We take a quaternion Gaussian G (m x r) and return its polar factor
Q = G (G^H G)^{-1/2}, computed in the complex-adjoint form (Section 2: the 2m x 2n complex
representation is an injective *-homomorphism, so the adjoint of the polar factor is the polar factor
of the adjoint).  Q spans the same column space as the Q factor of a quaternion QR of G; the two
differ by an r x r unitary right factor that depends on G, so both are Haar-distributed on the
quaternion Stiefel manifold and A = U diag(s) V^H has the same distribution either way.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian", "stiefel", "from_factors", "geometric", "round_f32",
    "c1_instance", "c2_instance", "c3_instance", "c4_sizes", "c4_instance",
    "c5_instance", "small_spectral_instance",
]


# ----------------------------------------------------------------------------------------------
# complex-adjoint helpers (local to the generator; the oracle has its own)
# ----------------------------------------------------------------------------------------------
def _to_cplx(P: np.ndarray) -> np.ndarray:
    """planes (4,m,n) -> complex adjoint (2m,2n) per Section 2's 2x2 block form."""
    a1 = P[0] + 1j * P[1]
    a2 = P[2] + 1j * P[3]
    return np.block([[a1, a2], [-np.conj(a2), np.conj(a1)]])


def _from_cplx(C: np.ndarray) -> np.ndarray:
    """complex adjoint (2m,2n) -> planes (4,m,n); averages the two copies of each block."""
    m, n = C.shape[0] // 2, C.shape[1] // 2
    a1 = 0.5 * (C[:m, :n] + np.conj(C[m:, n:]))
    a2 = 0.5 * (C[:m, n:] - np.conj(C[m:, :n]))
    return np.stack([a1.real, a1.imag, a2.real, a2.imag])


# ----------------------------------------------------------------------------------------------
# primitives
# ----------------------------------------------------------------------------------------------
def gaussian(seed: int, m: int, n: int) -> np.ndarray:
    """(4,m,n) planes, each component iid N(0,1), NumPy PCG64 stream `seed`."""
    return np.random.default_rng(seed).standard_normal((4, m, n))


def stiefel(seed: int, m: int, r: int) -> np.ndarray:
    """m x r quaternion matrix with orthonormal columns (U^H U = I_r): polar factor of a Gaussian."""
    if r > m:
        raise ValueError("stiefel: r must be <= m")
    Gc = _to_cplx(gaussian(seed, m, r))
    M = Gc.conj().T @ Gc
    w, W = np.linalg.eigh(M)
    Qc = Gc @ ((W / np.sqrt(w)) @ W.conj().T)
    return _from_cplx(Qc)


def householder_unitary(seed: int, n: int, k: int = 64) -> np.ndarray:
    """n x n unitary quaternion matrix: the product of k quaternion Householder reflectors
    H = I - 2 v v^H / (v^H v), v with iid N(0,1) components.  Built in the complex-adjoint form, where a
    reflector is the rank-2 update I - 2 chi(v) chi(v)^H / ||v||^2 (O(n^2) each), so large factors cost
    seconds instead of an O(n^3) orthonormalisation.  Used for square matrices with a prescribed spectrum."""
    rng = np.random.default_rng(seed)
    Q = np.eye(2 * n, dtype=np.complex128)
    for _ in range(k):
        v = rng.standard_normal((4, n, 1))
        vc = _to_cplx(v)  # 2n x 2
        nv2 = float(np.sum(v * v))
        Q -= (2.0 / nv2) * (Q @ vc) @ vc.conj().T
    return _from_cplx(Q)


def from_factors(U: np.ndarray, s: np.ndarray, V: np.ndarray) -> np.ndarray:
    """A = U diag(s) V^H for U (4,m,r), real s (r,), V (4,n,r) -> planes (4,m,n)."""
    Uc, Vc = _to_cplx(U), _to_cplx(V)
    s2 = np.concatenate([s, s])
    return _from_cplx((Uc * s2) @ Vc.conj().T)


def geometric(r: int, hi: float, lo: float) -> np.ndarray:
    """s_i = hi * (lo/hi)^((i-1)/(r-1)), i = 1..r (geometric spectrum from hi down to lo)."""
    if r == 1:
        return np.array([hi], dtype=np.float64)
    t = np.arange(r, dtype=np.float64) / (r - 1)
    return hi * (lo / hi) ** t


def round_f32(A: np.ndarray) -> np.ndarray:
    """Round to the nearest float32 and widen back (the FP32 instance, as the oracle sees it)."""
    return A.astype(np.float32).astype(np.float64)


def _cond(P: np.ndarray) -> float:
    sv = np.linalg.svd(_to_cplx(P), compute_uv=False)
    r = min(P.shape[1], P.shape[2])
    # every singular value of A appears twice in the adjoint
    return float(sv[0] / sv[2 * r - 1])


# ----------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------
def c1_instance(seed: int = 0, m: int = 64, n: int = 48) -> np.ndarray:
    """Small dense case: 64 x 48, planes iid N(0,1), seeds 0..9 (full column rank w.p. 1)."""
    return gaussian(seed, m, n)


def c2_instance(m: int = 2048, n: int = 1536, r: int = 1024, seeds=(100, 101),
                smin: float = 1e-4) -> dict:
    """Rank-r tall case: A = U diag(s) V^H, s geometric 1 -> smin, factors from Gaussians.

    Built in float64 and rounded to float32; ``A`` holds the float32 values widened to float64.
    """
    U = stiefel(seeds[0], m, r)
    V = stiefel(seeds[1], n, r)
    s = geometric(r, 1.0, smin)
    A64 = from_factors(U, s, V)
    return {"A": round_f32(A64), "A64": A64, "U": U, "s": s, "V": V}


def c3_instance(n: int = 4096, seeds=(200, 201), cond: float = 1e3, reflectors: int = 64) -> dict:
    """Square case with condition number `cond`, geometric spectrum, component variance ~1.

    Factors are products of `reflectors` random quaternion Householder reflectors (see
    householder_unitary).  c = 2n / sqrt(sum s_i^2) makes the mean squared component
    c^2 sum s^2 / (4 n^2) equal to 1.
    """
    U = householder_unitary(seeds[0], n, reflectors)
    V = householder_unitary(seeds[1], n, reflectors)
    s = geometric(n, 1.0, 1.0 / cond)
    c = 2.0 * n / np.sqrt(np.sum(s * s))
    s = c * s
    A64 = from_factors(U, s, V)
    return {"A": round_f32(A64), "A64": A64, "U": U, "s": s, "V": V}


def c4_sizes(count: int = 512, lo: int = 32, hi: int = 256, seed: int = 300) -> np.ndarray:
    """(count, 2) int array of (rows, cols), each iid uniform on [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=(count, 2))


def c4_instance(b: int, sizes: np.ndarray, seed0: int = 300, max_cond: float = 1e3) -> np.ndarray:
    """Matrix b of the batched workload: planes iid N(0,1), resampled (seed + 1000) while cond > max_cond."""
    m, n = int(sizes[b, 0]), int(sizes[b, 1])
    seed = seed0 + b
    while True:
        A = gaussian(seed, m, n)
        if _cond(A) <= max_cond:
            return A
        seed += 1000


def c5_instance(seed: int, m: int, n: int, family: str) -> dict:
    """One learned-scaling matrix: spectrum family in {geometric, clustered, lowrank}.

    geometric: s_i = kappa^(-(i-1)/(r-1)), log10 kappa ~ U[1,4].
    clustered: 2..5 levels 10^-U[0,3] (top level 1); each s_i takes a uniform level, +-1% log-normal jitter.
    lowrank:   rank k ~ U{2..floor(r/4)} with values 10^-U[0,1] (top 1) plus a Gaussian E whose
               planes have std 1e-3 / (2 (sqrt m + sqrt n)), so ||E||_2 ~ 1e-3; such instances are
               returned with ``s = None`` (the spectrum is only known after the noise is added).
    """
    rng = np.random.default_rng(seed)
    r = min(m, n)
    U = stiefel(seed * 2 + 1, m, r)
    V = stiefel(seed * 2 + 2, n, r)
    if family == "geometric":
        kappa = 10.0 ** rng.uniform(1.0, 4.0)
        s = geometric(r, 1.0, 1.0 / kappa)
        return {"A": from_factors(U, s, V), "s": s, "family": family}
    if family == "clustered":
        c = int(rng.integers(2, 6))
        levels = np.concatenate([[1.0], 10.0 ** (-rng.uniform(0.0, 3.0, size=c - 1))])
        idx = rng.integers(0, c, size=r)
        idx[0] = 0
        s = levels[idx] * np.exp(0.01 * rng.standard_normal(r))
        s = np.sort(s)[::-1]
        return {"A": from_factors(U, s, V), "s": s, "family": family}
    if family == "lowrank":
        k = int(rng.integers(2, max(3, r // 4 + 1)))
        sv = np.sort(10.0 ** (-rng.uniform(0.0, 1.0, size=k)))[::-1]
        sv[0] = 1.0
        s = np.zeros(r)
        s[:k] = sv
        L = from_factors(U, s, V)
        sig_e = 1e-3 / (2.0 * (np.sqrt(m) + np.sqrt(n)))
        E = sig_e * rng.standard_normal((4, m, n))
        return {"A": L + E, "s": None, "family": family}
    raise ValueError(f"unknown family {family!r}")


def small_spectral_instance(seed: int, m: int, n: int, s: np.ndarray) -> dict:
    """A = U diag(s) V^H with len(s) = r <= min(m,n), factors from Gaussians (seeds 2*seed+1, 2*seed+2)."""
    r = len(s)
    U = stiefel(2 * seed + 1, m, r)
    V = stiefel(2 * seed + 2, n, r)
    return {"A": from_factors(U, np.asarray(s, dtype=np.float64), V), "U": U, "s": np.asarray(s), "V": V}
