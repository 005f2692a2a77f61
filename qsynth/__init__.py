"""Seeded synthetic quaternion inputs, shared by the GPU path's tests/benchmarks and the CPU oracle.

This module only *builds inputs*: Gaussian component planes, prescribed singular-value spectra and
orthonormal quaternion factors, and the product A = U diag(s) V^H that places a spectrum on them.
It holds none of the pseudoinverse method's arithmetic (no residuals, no hyperpower polynomials,
no scaling rule) and imports neither the oracle nor the GPU package.

Storage convention (both sides): a quaternion matrix A = A_s + A_x i + A_y j + A_z k of shape m x n is
a float64 array of shape (4, m, n), planes in the order (s, x, y, z).

Construction of orthonormal quaternion factors.  The paper's experiments use unseeded Gaussian
matrices (Section 4).  For matrices with a prescribed spectrum we need quaternion matrices with
orthonormal columns.
  * stiefel(): the polar factor Q = G (G^H G)^{-1/2} of a quaternion Gaussian G (m x r), computed in the
    complex-adjoint form (Section 2: the 2m x 2n complex representation is an injective
    *-homomorphism, so the adjoint of the polar factor is the polar factor of the adjoint).  Q spans
    the same column space as the Q factor of a quaternion QR of G; the two differ by an r x r unitary
    right factor that depends on G, so both are Haar-distributed on the quaternion Stiefel manifold and
    A = U diag(s) V^H has the same distribution either way.  O(m r^2); used for the 2048 x 1536 case.
  * StructuredUnitary: U = C D_1 C D_2 C D_3 (orthonormal DCT-II and diagonals of random unit
    quaternions), dense and applied in O(n^2 log n); used where an O(n^3) factor is too slow (the
    4096 x 4096 case and the thousands of learned-scaling matrices).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian", "stiefel", "from_factors", "geometric", "round_f32", "StructuredUnitary",
    "structured_spectral", "structured_pinv", "mp_quantiles",
    "c1_instance", "c2_instance", "c3_instance", "c4_sizes", "c4_instance",
    "c5_spectrum", "c5_sample", "small_spectral_instance",
    "lorenz_trajectory", "lorenz_filter_instance", "LORENZ_STEPS", "cur_image_instance", "krylov_instance",
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


def low_rank_gaussian(seed: int, m: int, n: int, r: int) -> np.ndarray:
    """(4,m,n) planes of G H, G (m x r) and H (r x n) with components iid N(0,1) (streams seed, seed + 1):
    rank r almost surely.  The product is formed through the complex adjoint (a homomorphism)."""
    G = gaussian(seed, m, r)
    H = gaussian(seed + 1, r, n)
    return _from_cplx(_to_cplx(G) @ _to_cplx(H))


def stiefel(seed: int, m: int, r: int) -> np.ndarray:
    """m x r quaternion matrix with orthonormal columns (U^H U = I_r): polar factor of a Gaussian."""
    if r > m:
        raise ValueError("stiefel: r must be <= m")
    Gc = _to_cplx(gaussian(seed, m, r))
    M = Gc.conj().T @ Gc
    w, W = np.linalg.eigh(M)
    Qc = Gc @ ((W / np.sqrt(w)) @ W.conj().T)
    return _from_cplx(Qc)


#: threads of the DCTs in StructuredUnitary (-1: all cores; a process pool sets 1 per worker)
DCT_WORKERS = -1


def _unit_quaternions(rng, n: int) -> np.ndarray:
    """(4, n) random unit quaternions (normalised Gaussian 4-vectors: uniform on the 3-sphere)."""
    q = rng.standard_normal((4, n))
    return q / np.sqrt(np.sum(q * q, axis=0, keepdims=True))


def _left_diag(q: np.ndarray, M: np.ndarray) -> np.ndarray:
    """diag(q) M: row i of the quaternion matrix M multiplied on the left by the quaternion q_i."""
    a = [q[t][:, None] for t in range(4)]
    b = M
    return np.stack([a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                     a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                     a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                     a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]])


def _conj(q: np.ndarray) -> np.ndarray:
    return np.stack([q[0], -q[1], -q[2], -q[3]])


class StructuredUnitary:
    """Dense random unitary U = C D_1 C D_2 C D_3 of order n: C is the orthonormal DCT-II (real, so it acts
    on each plane), D_i = diag of random unit quaternions.  U and U^H are applied to quaternion matrices in
    O(n^2 log n) without forming U; for square matrices with a prescribed spectrum at sizes where an
    O(n^3) orthonormalisation is too slow."""

    def __init__(self, seed: int, n: int, rounds: int = 3):
        rng = np.random.default_rng(seed)
        self.n = n
        self.d = [_unit_quaternions(rng, n) for _ in range(rounds)]

    @staticmethod
    def _dct(M: np.ndarray, inverse: bool) -> np.ndarray:
        from scipy.fft import dct, idct

        return (idct if inverse else dct)(M, type=2, norm="ortho", axis=1, workers=DCT_WORKERS)

    def apply(self, M: np.ndarray) -> np.ndarray:
        """U M (M is n x k)."""
        for q in reversed(self.d):
            M = self._dct(_left_diag(q, M), inverse=True)
        return M

    def apply_h(self, M: np.ndarray) -> np.ndarray:
        """U^H M."""
        for q in self.d:
            M = _left_diag(_conj(q), self._dct(M, inverse=False))
        return M


def _qh(M: np.ndarray) -> np.ndarray:
    return np.stack([M[0].T, -M[1].T, -M[2].T, -M[3].T])


def structured_spectral(seeds, m: int, n: int, s: np.ndarray) -> np.ndarray:
    """A = U [diag(s) 0; 0 0] V^H with U (m x m), V (n x n) structured random unitaries; len(s) <= min(m, n)."""
    U = StructuredUnitary(seeds[0], m)
    V = StructuredUnitary(seeds[1], n)
    S = np.zeros((4, m, n))
    r = len(s)
    S[0, np.arange(r), np.arange(r)] = s
    # A = U S V^H = U (V S^H)^H
    return U.apply(_qh(V.apply(_qh(S))))


def structured_pinv(seeds, m: int, n: int, s: np.ndarray) -> np.ndarray:
    """The pseudoinverse V [diag(1/s) 0; 0 0] U^H of structured_spectral(seeds, m, n, s)."""
    U = StructuredUnitary(seeds[0], m)
    V = StructuredUnitary(seeds[1], n)
    S = np.zeros((4, n, m))
    r = len(s)
    S[0, np.arange(r), np.arange(r)] = 1.0 / np.asarray(s)
    return V.apply(_qh(U.apply(_qh(S))))


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


def c3_instance(n: int = 4096, seeds=(200, 201), cond: float = 1e3) -> dict:
    """Square case with condition number `cond`, geometric spectrum, component variance ~1.

    A = U diag(s) V^H with structured random unitaries (StructuredUnitary); c = 2n / sqrt(sum s_i^2)
    makes the mean squared component c^2 sum s^2 / (4 n^2) equal to 1.  ``seeds`` name the factors
    (the pseudoinverse is structured_pinv(seeds, n, n, s)).
    """
    s = geometric(n, 1.0, 1.0 / cond)
    c = 2.0 * n / np.sqrt(np.sum(s * s))
    s = c * s
    A64 = structured_spectral(seeds, n, n, s)
    return {"A": round_f32(A64), "A64": A64, "s": s, "seeds": tuple(seeds)}


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


def mp_quantiles(count: int, m: int, n: int, scale: float) -> np.ndarray:
    """`count` singular values at the midpoint quantiles of the Marchenko--Pastur law of an m x n matrix
    whose entries have variance scale^2 (support scale (sqrt M -+ sqrt N), M = max, N = min), descending."""
    M, N = max(m, n), min(m, n)
    c = N / M
    lo, hi = (1 - np.sqrt(c)) ** 2, (1 + np.sqrt(c)) ** 2
    x = np.linspace(lo, hi, 20001)
    dens = np.sqrt(np.clip((hi - x) * (x - lo), 0, None)) / x
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(x))])
    cdf /= cdf[-1]
    q = (np.arange(count) + 0.5) / count
    lam = np.interp(q, cdf, x)  # eigenvalues of W W^H / M
    return np.sort(scale * np.sqrt(M * lam))[::-1]


C5_FAMILIES = ("geometric", "clustered", "lowrank")


def c5_spectrum(seed: int, m: int, n: int, family: str) -> np.ndarray:
    """Singular values (descending, length min(m, n)) of one learned-scaling matrix.

    geometric: s_i = kappa^(-(i-1)/(r-1)), log10 kappa ~ U[1,4].
    clustered: 2..5 levels 10^-U[0,3] (top level 1); each s_i takes a uniform level, +-1% log-normal jitter.
    lowrank:   k ~ U{2..floor(r/4)} values 10^-U[0,1] (top 1) over a noise floor: the singular values of
               an m x n quaternion Gaussian with component std 1e-3 / (2 (sqrt m + sqrt n)) (so its norm
               is about 1e-3), taken at their Marchenko--Pastur quantiles.
    """
    rng = np.random.default_rng(seed)
    r = min(m, n)
    if family == "geometric":
        kappa = 10.0 ** rng.uniform(1.0, 4.0)
        return geometric(r, 1.0, 1.0 / kappa)
    if family == "clustered":
        c = int(rng.integers(2, 6))
        levels = np.concatenate([[1.0], 10.0 ** (-rng.uniform(0.0, 3.0, size=c - 1))])
        idx = rng.integers(0, c, size=r)
        idx[0] = 0
        s = levels[idx] * np.exp(0.01 * rng.standard_normal(r))
        return np.sort(s)[::-1]
    if family == "lowrank":
        k = int(rng.integers(2, max(3, r // 4 + 1)))
        sv = np.sort(10.0 ** (-rng.uniform(0.0, 1.0, size=k)))[::-1]
        sv[0] = 1.0
        sig_e = 1e-3 / (2.0 * (np.sqrt(m) + np.sqrt(n)))
        noise = mp_quantiles(r - k, m, n, 2.0 * sig_e) if r > k else np.zeros(0)
        return np.concatenate([sv, noise])
    raise ValueError(f"unknown family {family!r}")


def c5_sample(seed: int, size_range=(64, 512), shape=None, max_cond: float = 1e5) -> dict:
    """One learned-scaling matrix A = U diag(s) V^H (structured random factors): family uniform over
    C5_FAMILIES, m, n iid uniform in size_range unless `shape` is given, redrawn (seed + 1000) while
    cond > max_cond.  Returns A (float64 planes), s, family, m, n."""
    t = 0
    while True:
        rng = np.random.default_rng(seed + 1000 * t)
        family = C5_FAMILIES[int(rng.integers(0, 3))]
        if shape is None:
            m, n = (int(v) for v in rng.integers(size_range[0], size_range[1] + 1, size=2))
        else:
            m, n = shape
        s = c5_spectrum(seed * 7 + 1000 * t + 3, m, n, family)
        if s[-1] > 0 and s[0] / s[-1] <= max_cond:
            A = structured_spectral((2 * seed + 1 + 1000 * t, 2 * seed + 2 + 1000 * t), m, n, s)
            return {"A": A, "s": s, "family": family, "m": m, "n": n}
        t += 1


def small_spectral_instance(seed: int, m: int, n: int, s: np.ndarray) -> dict:
    """A = U diag(s) V^H with len(s) = r <= min(m,n), factors from Gaussians (seeds 2*seed+1, 2*seed+2)."""
    r = len(s)
    U = stiefel(2 * seed + 1, m, r)
    V = stiefel(2 * seed + 2, n, r)
    return {"A": from_factors(U, np.asarray(s, dtype=np.float64), V), "U": U, "s": np.asarray(s), "V": V}


# ----------------------------------------------------------------------------------------------
# Lorenz filtering workload (Section 5.2): a delayed, noisy quaternion observation of a Lorenz
# trajectory and the square Toeplitz data matrix of the filter design X h = s
# ----------------------------------------------------------------------------------------------
LORENZ_STEPS = (0.01, 0.02, 0.03, 0.04, 0.05)  # the sampling steps of the paper's filtering table


def lorenz_trajectory(T: float, dt: float, x0=(1.0, 1.0, 1.0), sigma: float = 10.0, delta: float = 8.0 / 3.0,
                      gamma: float = 28.0, sub: int = 10) -> np.ndarray:
    """(u, v, w) of the Lorenz system (Section 5.2: du/dt = sigma (v - u), dv/dt = u (gamma - w) - v,
    dw/dt = u v - delta w) at t = 0, dt, ..., round(T/dt) dt, from x0 at t = 0.  Classical fourth-order
    Runge-Kutta with `sub` steps per sample (the paper used an adaptive solver; the trajectory is
    chaotic, so sample values depend on the integrator beyond t ~ 20 either way).  Shape (n + 1, 3)."""
    n = int(round(T / dt))
    h = dt / sub

    def f(u, v, w):
        return sigma * (v - u), u * (gamma - w) - v, u * v - delta * w

    u, v, w = (float(c) for c in x0)
    out = np.empty((n + 1, 3))
    out[0] = (u, v, w)
    for k in range(n):
        for _ in range(sub):
            a = f(u, v, w)
            b = f(u + 0.5 * h * a[0], v + 0.5 * h * a[1], w + 0.5 * h * a[2])
            c = f(u + 0.5 * h * b[0], v + 0.5 * h * b[1], w + 0.5 * h * b[2])
            d = f(u + h * c[0], v + h * c[1], w + h * c[2])
            u += h / 6.0 * (a[0] + 2.0 * b[0] + 2.0 * c[0] + d[0])
            v += h / 6.0 * (a[1] + 2.0 * b[1] + 2.0 * c[1] + d[1])
            w += h / 6.0 * (a[2] + 2.0 * b[2] + 2.0 * c[2] + d[2])
        out[k + 1] = (u, v, w)
    return out


def lorenz_filter_instance(dt: float, T: float = 40.0, tau: float = 1.0, noise: float = 1.0,
                           seed: int = 500) -> dict:
    """Filter-design system of Section 5.2 for sampling step dt on [0, T].

    Samples k = 0..n (n = round(T/dt)).  Reference s_k = u_k i + v_k j + w_k k (pure quaternion).
    Observation x_k = s_{k-d} + eta_k with d = round(tau/dt) (held at s_0 before the record starts) and
    eta_k purely imaginary, iid N(0, noise^2) per imaginary component (PCG64 stream `seed`).  With
    p = n // 2, the data matrix is the (p+1) x (p+1) Toeplitz X[i, j] = x_{p+i-j} (first row x_p, x_{p-1},
    ..., x_0; last row x_{2p}, ..., x_p) and the target s = (s_p, ..., s_{2p}).
    Returns X (4, p+1, p+1), s (4, p+1, 1), x (4, n+1), ref (4, n+1) and the sizes."""
    traj = lorenz_trajectory(T, dt)
    n = traj.shape[0] - 1
    d = int(round(tau / dt))
    ref = np.zeros((4, n + 1))
    ref[1:] = traj.T
    rng = np.random.default_rng(seed)
    x = np.zeros((4, n + 1))
    x[1:] = ref[1:, np.maximum(np.arange(n + 1) - d, 0)] + noise * rng.standard_normal((3, n + 1))
    p = n // 2
    i = np.arange(p + 1)
    X = np.ascontiguousarray(x[:, p + i[:, None] - i[None, :]])
    s = np.ascontiguousarray(ref[:, p:2 * p + 1, None])
    return {"X": X, "s": s, "x": x, "ref": ref, "p": p, "delay": d, "dt": dt, "T": T}


# ----------------------------------------------------------------------------------------------
# CUR image completion workload (Section 5.1) on a synthetic colour image (the paper's Kodak image is
# not available): pure-quaternion pixels (0, R, G, B), a random mask of observed pixels and the row /
# column index sets of the CUR factors
# ----------------------------------------------------------------------------------------------
def cur_image_instance(m: int = 512, n: int = 768, terms: int = 40, texture: float = 0.02, missing: float = 0.7,
                       rank: int = 60, seed: int = 600) -> dict:
    """Image = 0.5 + sum of `terms` separable smooth patterns f_k(y) g_k(x) with random colour weights
    (each f, g a sum of 3 sinusoids of random low frequency and phase), scaled to a 0.35 amplitude per
    channel, plus iid N(0, texture^2) per channel.  Mask: each pixel observed with probability
    1 - missing.  rows / cols: `rank` distinct indices each, uniform, sorted.
    Returns image (4, m, n) with plane 0 zero, mask (m, n) uint8, rows, cols (int32)."""
    rng = np.random.default_rng(seed)
    y = np.linspace(0.0, 1.0, m)[:, None]
    x = np.linspace(0.0, 1.0, n)[None, :]

    def smooth(t, k):
        f = np.zeros_like(t)
        for _ in range(3):
            f = f + rng.standard_normal() * np.sin(2.0 * np.pi * (rng.uniform(0.2, 1.0 + 0.25 * k) * t + rng.uniform()))
        return f

    img = np.zeros((4, m, n))
    for k in range(terms):
        pat = smooth(y, k) * smooth(x, k)
        w = rng.standard_normal(3) / (1.0 + k)
        for c in range(3):
            img[1 + c] += w[c] * pat
    for c in range(3):
        img[1 + c] *= 0.35 / max(np.abs(img[1 + c]).max(), 1e-12)
    img[1:] += 0.5 + texture * rng.standard_normal((3, m, n))
    mask = (rng.uniform(size=(m, n)) >= missing).astype(np.uint8)
    rows = np.sort(rng.choice(m, size=rank, replace=False)).astype(np.int32)
    cols = np.sort(rng.choice(n, size=rank, replace=False)).astype(np.int32)
    return {"image": img, "mask": mask, "rows": rows, "cols": cols}


# ----------------------------------------------------------------------------------------------
# Preconditioned Krylov workload (Section 4, Example 4): A = A_s (1 - i + 2 j + 1.5 k) with a real
# nonsymmetric A_s standing in for the 238 x 238 Matrix-Market matrix the paper uses (not available)
# ----------------------------------------------------------------------------------------------
def krylov_instance(m: int, grid=(14, 17), contrast: float = 2.0, convection: float = 0.5, shift: float = 1e-3,
                    seed: int = 700) -> dict:
    """A_s: a five-point finite-volume operator on a grid[0] x grid[1] mesh (n = 238 by default, the
    size of the paper's matrix) with log-normal transmissibilities exp(contrast N(0,1)) on the mesh
    edges, a skew (convective) part convection * t * N(0,1) on the same edges, and a diagonal
    accumulation term shift * mean(t).  The quaternion coefficient matrix follows Example 4:
    A^(x) = -A_s, A^(y) = 2 A_s, A^(z) = 1.5 A_s.  B: n x m, every plane iid uniform [0, 1)."""
    rng = np.random.default_rng(seed)
    nx, ny = grid
    n = nx * ny
    As = np.zeros((n, n))
    ts = []
    for i in range(nx):
        for j in range(ny):
            a = i * ny + j
            for b in ([a + ny] if i + 1 < nx else []) + ([a + 1] if j + 1 < ny else []):
                t = float(np.exp(contrast * rng.standard_normal()))
                u = convection * t * float(rng.standard_normal())
                ts.append(t)
                As[a, a] += t
                As[b, b] += t
                As[a, b] += -t + u
                As[b, a] += -t - u
    As += shift * float(np.mean(ts)) * np.eye(n)
    A = np.stack([As, -As, 2.0 * As, 1.5 * As])
    B = rng.uniform(size=(4, n, m))
    return {"A": A, "B": B, "As": As}
