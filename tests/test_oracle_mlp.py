"""Pins of the FP64 learned-start network: finite differences, invariances, Adam's first step."""
import numpy as np
import pytest

from oracle import mlp, sym


def _setup(seed=0, B=7, K=28):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng, K)
    for k in ("b1", "b2", "b3"):
        p[k] = 0.1 * rng.standard_normal(p[k].shape)
    C = rng.standard_normal((B, K))
    X = mlp.features(C, 6)
    t = rng.standard_normal((B, 3))
    return p, X, t


def test_features_are_orthonormal_coordinates():
    rng = np.random.default_rng(1)
    C = rng.standard_normal((5, 28))
    X = mlp.features(C, 6)
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0)
    # |x| = 1 because ||C||_F^2 = sum mu_a C_a^2
    assert np.allclose(np.linalg.norm(C * np.sqrt(sym.weights(6, 3)), axis=1), sym.frobenius(C.T, 6, 3))
    assert np.all(mlp.features(np.zeros((1, 28)), 6) == 0)


def test_gradients_match_finite_differences():
    p, X, t = _setup()
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, t)
    h = 1e-6
    rng = np.random.default_rng(2)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], t)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert fd == pytest.approx(g[k].reshape(-1)[idx], rel=1e-5, abs=1e-9), k


def test_loss_sign_invariant_and_bounded():
    p, X, t = _setup(3)
    y, _ = mlp.forward(p, X)
    l0 = mlp.loss(y, t)
    assert 0.0 <= l0 <= 1.0
    assert mlp.loss(y, -t) == pytest.approx(l0)
    assert mlp.loss(-y, t) == pytest.approx(l0)
    assert mlp.loss(t * 3.0, t) == pytest.approx(0.0, abs=1e-15)


def test_adam_first_step_closed_form():
    # with bias correction the first Adam step is -lr * g / (|g| + eps) elementwise
    p, X, t = _setup(4)
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, t)
    p0 = {k: v.copy() for k, v in p.items()}
    st = mlp.adam_init(p)
    mlp.adam_step(p, g, st, lr=1e-2, eps=1e-8)
    for k in p:
        assert np.allclose(p[k], p0[k] - 1e-2 * g[k] / (np.abs(g[k]) + 1e-8), atol=1e-12)


def test_training_reduces_loss_on_a_learnable_map():
    rng = np.random.default_rng(5)
    B = 256
    v = rng.standard_normal((B, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    C = sym.monomials(v, 6) + 0.05 * rng.standard_normal((B, 28))   # rank one + noise
    X = mlp.features(C, 6)
    p = mlp.init_params(rng, 28)
    st = mlp.adam_init(p)
    l0 = mlp.loss(mlp.forward(p, X)[0], v)
    for _ in range(300):
        y, cache = mlp.forward(p, X)
        mlp.adam_step(p, mlp.backward(p, cache, v), st, lr=3e-3)
    l1 = mlp.loss(mlp.forward(p, X)[0], v)
    assert l1 < 0.2 * l0


def test_bf16_round_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.140625, 1e-3])
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie: rounds to even mantissa
    assert r[2] == 1.0 + 2 ** -7            # above the tie: rounds up
    assert r[3] == -2.5 and r[4] == 3.140625
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8
