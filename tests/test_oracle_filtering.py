"""Filter design of Section 5.2: the Lorenz input generator and the oracle's h = X^dagger s, pinned
against an independent integrator, an exact equilibrium, a linear solve, the normal equations and a
constructed pseudoinverse."""
import numpy as np
import pytest

import qsynth
from oracle import filtering as F
from oracle import quat as Q

U64 = np.finfo(np.float64).eps


def test_lorenz_rk4_matches_an_independent_integrator():
    """Before chaos amplifies rounding (t <= 1), the generator's RK4 agrees with SciPy's DOP853."""
    from scipy.integrate import solve_ivp

    sigma, delta, gamma = 10.0, 8.0 / 3.0, 28.0

    def f(t, y):
        return [sigma * (y[1] - y[0]), y[0] * (gamma - y[2]) - y[1], y[0] * y[1] - delta * y[2]]

    traj = qsynth.lorenz_trajectory(1.0, 0.01)
    ref = solve_ivp(f, (0.0, 1.0), [1.0, 1.0, 1.0], method="DOP853", rtol=1e-12, atol=1e-12,
                    t_eval=np.linspace(0.0, 1.0, 101))
    assert np.max(np.abs(traj - ref.y.T)) <= 1e-7


def test_lorenz_equilibrium_is_fixed():
    """(sqrt(delta (gamma - 1)), sqrt(delta (gamma - 1)), gamma - 1) is an equilibrium of the system."""
    delta, gamma = 8.0 / 3.0, 28.0
    c = np.sqrt(delta * (gamma - 1.0))
    traj = qsynth.lorenz_trajectory(0.5, 0.05, x0=(c, c, gamma - 1.0))
    assert np.max(np.abs(traj - traj[0])) <= 1e-11


def test_filter_instance_layout():
    d = qsynth.lorenz_filter_instance(0.05, T=8.0)
    X, s, x, ref, p, dd = d["X"], d["s"], d["x"], d["ref"], d["p"], d["delay"]
    n = x.shape[1] - 1
    assert n == 160 and p == 80 and dd == 20 and X.shape == (4, p + 1, p + 1) and s.shape == (4, p + 1, 1)
    assert F.toeplitz_columns(X)
    assert np.array_equal(X[:, 0, :], x[:, p::-1])  # first row x_p, ..., x_0
    assert np.array_equal(X[:, :, 0], x[:, p:2 * p + 1])  # first column x_p, ..., x_2p
    assert np.array_equal(s[:, :, 0], ref[:, p:2 * p + 1])
    assert not X[0].any() and not s[0].any()  # pure quaternions
    # the observation is the delayed reference plus noise: the noise has the stated scale
    eta = x[1:, dd:] - ref[1:, :n + 1 - dd]
    assert 0.8 <= eta.std() <= 1.2


def test_design_invertible_matches_a_linear_solve():
    """Square invertible X: h = X^{-1} s (solved in the complex adjoint) and eps ~ machine precision."""
    X = qsynth.gaussian(7, 40, 40)
    s = qsynth.gaussian(8, 40, 1)
    out = F.design(X, s)
    h_solve = F.design_invertible(X, s)["h"]
    kappa = Q.sigma_max(X) / Q.singular_values(X)[-1]
    assert Q.fro(out["h"] - h_solve) <= 100 * kappa * U64 * Q.fro(h_solve)
    assert out["eps"] <= 100 * kappa * U64


def test_design_tall_satisfies_normal_equations():
    """Overdetermined X (full column rank): X^H (X h - s) = 0 and eps equals the least-squares residual."""
    X = qsynth.gaussian(9, 60, 25)
    s = qsynth.gaussian(10, 60, 1)
    out = F.design(X, s)
    g = Q.qmul(Q.qH(X), out["s_hat"] - s)
    assert Q.fro(g) <= 1e-12 * Q.fro(X) * Q.fro(s)
    h_ne = Q.qmul(Q.pinv_full_column_rank(X), s)
    assert Q.fro(out["h"] - h_ne) <= 1e-10 * Q.fro(h_ne)
    assert 0.1 < out["eps"] < 1.0


def test_design_rank_deficient_uses_the_constructed_pseudoinverse():
    inst = qsynth.small_spectral_instance(11, 30, 30, np.array([3.0, 2.0, 1.0, 0.5]))
    s = qsynth.gaussian(12, 30, 1)
    out = F.design(inst["A"], s)
    h_ref = Q.qmul(Q.pinv_from_factors(inst["U"], inst["s"], inst["V"]), s)
    assert Q.fro(out["h"] - h_ref) <= 1e-12 * Q.fro(h_ref)


@pytest.mark.parametrize("dt", [0.05, 0.04])
def test_small_lorenz_design_recovers_the_target(dt):
    """On a short record the Toeplitz system is square and invertible: eps is bounded by its condition."""
    d = qsynth.lorenz_filter_instance(dt, T=8.0)
    out = F.design(d["X"], d["s"])
    sv = Q.singular_values(d["X"])
    assert out["eps"] <= 1e3 * (sv[0] / sv[-1]) * U64
