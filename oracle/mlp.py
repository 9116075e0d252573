"""FP64 reference of the learned start for the orientation search.  TEST INFRASTRUCTURE ONLY.

The paper seeds SS-HOPM from an iterative eigendecomposition plus many
uniform starts (Sec. 3.1).  The learned start replaces those seeds by a small
network that maps the voxel's tensor to a direction:

    x   = (sqrt(mu_a) C_a) / ||C||_F           (orthonormal coordinates, |x| = 1)
    h1  = relu(x W1 + b1)                       K -> 64
    h2  = relu(h1 W2 + b2)                      64 -> 64
    y   = h2 W3 + b3                            64 -> d'
    u   = y / |y|

trained with the sign-invariant loss 1 - (u . t)^2 against target directions
t (the multistart answers), and Adam.  Everything here is plain FP64 numpy,
forward and backward written out by hand.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss for
every parameter; the loss is invariant under t -> -t and y -> -y and lies in
[0, 1]; one Adam step against the closed form of its first step.
"""
from __future__ import annotations

import numpy as np

from . import sym

HIDDEN = 64


def init_params(rng: np.random.Generator, k_in: int, d_out: int = 3, hidden: int = HIDDEN) -> dict:
    """He-normal weights, zero biases."""
    return {
        "W1": rng.standard_normal((k_in, hidden)) * np.sqrt(2.0 / k_in),
        "b1": np.zeros(hidden),
        "W2": rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden),
        "b2": np.zeros(hidden),
        "W3": rng.standard_normal((hidden, d_out)) * np.sqrt(1.0 / hidden),
        "b3": np.zeros(d_out),
    }


def features(C: np.ndarray, n: int, d: int = 3) -> np.ndarray:
    """x = sqrt(mu_a) C_a / ||C||_F for C of shape (B, K); zero tensors map to 0."""
    C = np.atleast_2d(np.asarray(C, dtype=np.float64))
    x = C * np.sqrt(sym.weights(n, d))[None, :]
    nrm = np.linalg.norm(x, axis=1, keepdims=True)
    return np.where(nrm > 0, x / np.where(nrm > 0, nrm, 1.0), 0.0)


def forward(p: dict, X: np.ndarray):
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (X, z1, h1, z2, h2, y)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    """mean over the batch of 1 - (y.t / |y||t|)^2."""
    u = y / np.linalg.norm(y, axis=1, keepdims=True)
    tt = t / np.linalg.norm(t, axis=1, keepdims=True)
    return float(np.mean(1.0 - np.sum(u * tt, axis=1) ** 2))


def backward(p: dict, cache, t: np.ndarray) -> dict:
    """Gradients of loss() with respect to every parameter."""
    X, z1, h1, z2, h2, y = cache
    B = X.shape[0]
    tt = t / np.linalg.norm(t, axis=1, keepdims=True)
    ny = np.linalg.norm(y, axis=1, keepdims=True)
    u = y / ny
    c = np.sum(u * tt, axis=1, keepdims=True)
    # L_b = 1 - c^2, c = u.t, u = y/|y|: dL/dy = -2c (t - c u) / |y|
    dy = (-2.0 * c * (tt - c * u) / ny) / B
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return g


def adam_init(p: dict) -> dict:
    return {"t": 0, "m": {k: np.zeros_like(v) for k, v in p.items()},
            "v": {k: np.zeros_like(v) for k, v in p.items()}}


def adam_step(p: dict, g: dict, st: dict, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """In-place Adam update (Kingma & Ba) with bias correction."""
    st["t"] += 1
    t = st["t"]
    for k in p:
        st["m"][k] = b1 * st["m"][k] + (1 - b1) * g[k]
        st["v"][k] = b2 * st["v"][k] + (1 - b2) * g[k] ** 2
        mh = st["m"][k] / (1 - b1 ** t)
        vh = st["v"][k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def predict(p: dict, C: np.ndarray, n: int, d: int = 3) -> np.ndarray:
    """Unit start directions for tensors C (B, K)."""
    y, _ = forward(p, features(C, n, d))
    return y / np.linalg.norm(y, axis=1, keepdims=True)
