"""The FP32 host evaluation used for FP32 parity bounds follows the same updates as the oracle (CPU only)."""
import numpy as np
import pytest

import fp32_chain as F32
import qsynth
from oracle import methods as M
from oracle import quat as Q


@pytest.mark.parametrize("method,order", [("ns", 2), ("qsai", 10), ("qhpi19", 19), ("qrapid", 5), ("qrapid", 1)])
def test_fp32_chain_tracks_oracle(method, order):
    """On a well-conditioned 40 x 30 matrix the FP32 evaluation stays within FP32 rounding of the oracle's
    iterates (a wrong coefficient or product order would be off by O(1)), and it does round (not exact)."""
    inst = qsynth.small_spectral_instance(5, 40, 30, qsynth.geometric(30, 1.0, 0.2))
    A = qsynth.round_f32(inst["A"])
    X0 = qsynth.round_f32(M.x0(A, 1.0 / Q.singular_values(A)[0] ** 2))
    Xo = X0
    for j in range(1, 4):
        Xo = M.step(A, Xo, method, order, "left")
        X32 = F32.iterate(A, X0, method, j, order)
        err = Q.fro(X32 - Xo) / Q.fro(Xo)
        assert 1e-9 < err <= 2e-6, (method, j, err)
    assert F32.iterate(A, X0, method, 1, order).dtype == np.float64
