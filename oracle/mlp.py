"""Float64 reference of the scaling network (oracle; test infrastructure only).

The network predicts y = log(mu), mu = alpha * sigma1_est^2, for X_0 = alpha A^H (Theorem 1).
Inputs are ten scale-invariant transforms of the raw scaling features
(sigma1_est^2, the previous power-step estimate, ||A||_F, ||A||_1, ||A||_inf, m, n), standardised
with stored means and deviations.  Two tanh hidden layers of width 64, linear output, mean squared
error.  Parameter layout (one flat vector): W1 (10 x 64, row-major), b1 (64), W2 (64 x 64), b2 (64),
W3 (64), b3 (1).

Pinned by central finite differences in the tests (no other reference exists: the network is not
part of the paper).
"""
from __future__ import annotations

import numpy as np

F, H = 10, 64
SIZES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def transform(raw: np.ndarray) -> np.ndarray:
    """raw rows (s1sq, s1sq_prev, fro, norm1, norminf, m, n) -> the ten network inputs."""
    s1, s1p, fro, n1, ni, m, n = (raw[:, k] for k in range(7))
    mn, mx = np.minimum(m, n), np.maximum(m, n)
    return np.stack([
        np.log(m), np.log(n), np.log(mn / mx),
        np.log(fro * fro / s1),
        np.log(n1 * ni / s1),
        np.log(n1 / ni),
        np.log(fro * fro / (s1 * mn)),
        s1p / s1,
        np.log(n1 / np.sqrt(m * s1)),
        np.log(ni / np.sqrt(n * s1)),
    ], axis=1)


def forward(theta, Z):
    """Z: standardised inputs (B x 10).  Returns y (B,) and the hidden activations."""
    p = unpack(theta)
    H1 = np.tanh(Z @ p["W1"] + p["b1"])
    H2 = np.tanh(H1 @ p["W2"] + p["b2"])
    y = H2 @ p["W3"] + p["b3"][0]
    return y, (H1, H2)


def loss_and_grad(theta, Z, t):
    """Mean squared error (1/B) sum (y - t)^2 and its gradient by backpropagation."""
    p = unpack(theta)
    B = Z.shape[0]
    y, (H1, H2) = forward(theta, Z)
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g["W3"] = H2.T @ dy
    g["b3"] = np.array([dy.sum()])
    d2 = np.outer(dy, p["W3"]) * (1.0 - H2 * H2)
    g["W2"] = H1.T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"].T) * (1.0 - H1 * H1)
    g["W1"] = Z.T @ d1
    g["b1"] = d1.sum(axis=0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SIZES])


def finite_difference_grad(theta, Z, t, h=1e-6):
    gd = np.zeros_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        lp, _ = loss_and_grad(theta + e, Z, t)
        lm, _ = loss_and_grad(theta - e, Z, t)
        gd[k] = (lp - lm) / (2 * h)
    return gd


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015), step counted from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
