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


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    Emulates the storage precision of the kernels' matrix-core operands.
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p: dict, X: np.ndarray, bf16: bool = False):
    """Forward pass; bf16=True rounds x, the weights and h1, h2 as the kernels store them."""
    r = bf16_round if bf16 else (lambda a: a)
    z1 = r(X) @ r(p["W1"]) + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(p["W2"]) + p["b2"]
    h2 = r(np.maximum(z2, 0.0))
    y = h2 @ r(p["W3"]) + p["b3"]
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


def padded_inputs(k_in: int) -> int:
    """Rows of W1 in the kernels' master layout: 32 for k_in <= 32, else 48."""
    return 32 if k_in <= 32 else 48


def pad_params(p: dict, k_in: int, d_out: int = 3) -> np.ndarray:
    """Flatten to the kernels' master layout: W1[kin][64] (kin = padded_inputs),
    b1[64], W2[64][64], b2[64], W3[64][16], b3[16] (padding rows / columns zero)."""
    W1 = np.zeros((padded_inputs(k_in), HIDDEN))
    W1[:k_in] = p["W1"]
    W3 = np.zeros((HIDDEN, 16))
    W3[:, :d_out] = p["W3"]
    b3 = np.zeros(16)
    b3[:d_out] = p["b3"]
    return np.concatenate([W1.ravel(), p["b1"], p["W2"].ravel(), p["b2"], W3.ravel(), b3])


def unpad_params(flat: np.ndarray, k_in: int, d_out: int = 3) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    o = 0
    kin = padded_inputs(k_in)
    W1 = flat[o:o + kin * HIDDEN].reshape(kin, HIDDEN)[:k_in]; o += kin * HIDDEN
    b1 = flat[o:o + HIDDEN]; o += HIDDEN
    W2 = flat[o:o + HIDDEN * HIDDEN].reshape(HIDDEN, HIDDEN); o += HIDDEN * HIDDEN
    b2 = flat[o:o + HIDDEN]; o += HIDDEN
    W3 = flat[o:o + HIDDEN * 16].reshape(HIDDEN, 16)[:, :d_out]; o += HIDDEN * 16
    b3 = flat[o:o + 16][:d_out]
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "W3": W3, "b3": b3}


def orient_learned(Cv: np.ndarray, n: int, p: dict, starts: np.ndarray, kappa: float,
                   tol: float = 1e-5, max_iter: int = 500, bf16: bool = True,
                   detail: bool = False, newton_first: int = 5, u0: np.ndarray | None = None,
                   polish: int = 2, certify: float = 1e-2):
    """Orientation with the learned start and its multistart fallback, for the
    axis form (d' = 3) and the quaternion form (d' = 4; d' is the starts'
    dimension, and the network has d' outputs).

    The learned start replaces the paper's seeds of SS-HOPM (Sec. 3.1); its
    search parameters (tol, max_iter, newton_first, polish, certify and the
    Newton search's drop rule) are part of that method's definition, since
    they decide which basin the answer comes from and whether the multistart
    runs:

    1. u0 = y / |y| from the network (fixed start 0 where y = 0, which also
       forces the fallback);
    2. up to ``newton_first`` Riemannian Newton steps (ttm.newton_ascent; the
       quaternion form's learned start takes none); if
       they do not converge, SS-HOPM from u0 with the unfolding shift until
       |delta lambda| <= tol or max_iter updates, then ``polish`` Newton steps
       (ttm.newton_polish); "converged" is the outcome of the search that ran
       last;
    3. the end point is certified near a local maximum (ttm.certify: the
       next Newton step is at most ``certify`` long, after at most four
       guarded Newton steps; a slow SS-HOPM run on a flat, curved ridge can
       meet its stopping rule far from the maximum);
    4. the learned answer is the converged maximum of the basin the search
       ended in (ttm.converge from its end point);
    5. fallback when the search did not converge, the end point is not
       certified, lambda / ||C||_F < kappa, or a fixed start s already has
       <C, s^n> > lambda (SS-HOPM never lowers lambda, so the multistart
       answer is then larger): the multistart answer (ttm.orient_multistart)
       is computed too and the larger lambda wins.

    Returns (lambda, u, fell_back), and with ``detail`` a fourth item: a dict
    with the learned answer (lam_learned, u_learned), how far each fallback
    test was from flipping (beat_gap = best fixed-start value minus the
    learned lambda, scaled by ||C||_F; kappa_gap = lambda / ||C||_F - kappa;
    cert_step = the last Newton step length the certification measured), whether the search
    converged, and after a fallback the multistart's per-start lambdas and
    directions.  ``u0`` (a unit vector) replaces the network's direction, to
    probe how the answer depends on the start.
    """
    from . import ttm
    starts = np.asarray(starts, dtype=np.float64)
    d = starts.shape[1]
    cn = float(sym.frobenius(Cv, n, d))
    if cn == 0.0:
        out = (0.0, np.zeros(d), False)
        return out + ({"lam_learned": 0.0, "u_learned": np.zeros(d), "beat_gap": -np.inf,
                       "kappa_gap": np.inf, "cert_step": 0.0, "converged": True, "lams": None,
                       "us": None},) if detail else out
    forced = False
    if u0 is None:
        y, _ = forward(p, features(Cv[None, :], n, d), bf16=bf16)
        y = y[0]
        ny = np.linalg.norm(y)
        forced = not ny > 0
        u0 = starts[0] / np.linalg.norm(starts[0]) if forced else y / ny
    Cu = np.asarray(Cv, dtype=np.float64) / cn
    alpha = ttm.unfolding_shift(Cu, n, d)
    u, lam, conv = ttm.newton_ascent(Cu, n, u0, newton_first, tol)
    if not conv:
        lam, u, _, conv = ttm.sshopm(Cu, n, u0, alpha, tol, max_iter)
        u = ttm.newton_polish(Cu, n, u, polish)
    u, certified, step = ttm.certify(Cu, n, u, certify)
    lam, u, _ = ttm.converge(Cu, n, u, alpha)
    fs = max(sym.inner_power(Cu, s / np.linalg.norm(s), n) for s in starts)
    beaten = fs > lam
    info = {"lam_learned": cn * lam, "u_learned": ttm.canonical_sign(u), "beat_gap": cn * (fs - lam),
            "kappa_gap": lam - kappa, "cert_step": step, "converged": conv, "lams": None, "us": None}
    if conv and certified and not forced and lam >= kappa and not beaten:
        out = (cn * lam, ttm.canonical_sign(u), False)
        return out + (info,) if detail else out
    lam_p, u_p, lams, us, _ = ttm.orient_multistart(Cv, n, starts)
    info["lams"], info["us"] = lams, us
    if lam_p > cn * lam:
        out = (lam_p, u_p, True)
    else:
        out = (cn * lam, ttm.canonical_sign(u), True)
    return out + (info,) if detail else out
