"""FP64 CPU oracle for the quaternion hyperpower pseudoinverse methods.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or executes this package:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
no code with the GPU path (no kernels, headers, helpers, tables or coefficient generators); both
sides only read inputs built by the separate ``qsynth`` generator module.

It is written to be plain and checkable against the paper by eye:

* ``quat``    -- quaternion algebra on (4, m, n) float64 planes: the 16-term Hamilton product
                 (Section 2), conjugate transpose, the complex adjoint, norms, and the plain
                 definitions of the Moore--Penrose inverse (SVD of the complex adjoint, closed
                 forms for full rank, V diag(1/s) U^H for constructed matrices).
* ``methods`` -- the iterations (Newton--Schulz, hyperpower HPI(p), QSAI Algorithm 2, QHPI19
                 Algorithm 3, QRAPID Algorithm 1) step by step in the paper's order, the scaling
                 rules, stop rules, Penrose residuals E1--E4 (Section 4) and the exact-arithmetic
                 spectral model of every iterate.
* ``mlp``     -- float64 forward/backward of the scaling network, for gradient checks.
* ``filtering`` -- the quaternion filter design of Section 5.2 (h = X^dagger s, s_hat = X h, eps).
* ``cur``     -- the CUR approximation and impute-reconstruct completion of Section 5.1.
* ``krylov``  -- global quaternion FOM / GMRES (Section 3.5, Example 4), plain and preconditioned.

Every function cites the passage it follows.  Functions whose result no independent pin checks are
marked "parity unpinned" in their docstring.
"""
from . import quat, methods, filtering, cur, krylov  # noqa: F401
