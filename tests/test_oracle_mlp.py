"""The float64 scaling-network reference against central finite differences (CPU)."""
import numpy as np

from oracle import mlp


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = 0.3 * rng.standard_normal(mlp.NPARAM)
    Z = rng.standard_normal((7, mlp.F))
    t = rng.standard_normal(7)
    _, g = mlp.loss_and_grad(theta, Z, t)
    gd = mlp.finite_difference_grad(theta, Z, t)
    assert np.max(np.abs(g - gd)) <= 1e-7 * max(1.0, np.max(np.abs(gd)))


def test_transform_is_scale_invariant():
    raw = np.array([[4.0, 3.9, 10.0, 20.0, 25.0, 300.0, 200.0]])
    c = 7.3  # A -> c A scales s1sq by c^2 and the norms by c
    raw2 = raw * np.array([[c * c, c * c, c, c, c, 1.0, 1.0]])
    np.testing.assert_allclose(mlp.transform(raw), mlp.transform(raw2), rtol=1e-12, atol=1e-12)


def test_adam_first_step_moves_by_lr():
    theta = np.zeros(3)
    g = np.array([1.0, -2.0, 0.5])
    th, m, v = mlp.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-6)
