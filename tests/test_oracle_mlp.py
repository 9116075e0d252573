"""Pins of the FP64 learned-start network: finite differences, invariances, Adam's first step."""
import math

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


# ---------------------------------------------------------------- the learned path's decisions
def _two_maxima(n=6, l1=2.0, l2=1.0, seed=3):
    """C = l1 a^n + l2 b^n with a, b, c orthonormal: <C, u^n> = l1 (a.u)^n + l2 (b.u)^n
    has local maxima l1 at +-a and l2 at +-b, its global maximum is max(l1, l2)
    (x^n + y^n <= x^2 + y^2 <= 1 on the sphere), and ||C||_F = sqrt(l1^2 + l2^2)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    a, b, c = Q[:, 0], Q[:, 1], Q[:, 2]
    C = l1 * sym.monomials(a, n) + l2 * sym.monomials(b, n)
    return C, a, b, c


def _tilt(u, w, deg):
    w = w - (w @ u) * u
    v = np.cos(np.radians(deg)) * u + np.sin(np.radians(deg)) * w / np.linalg.norm(w)
    return v / np.linalg.norm(v)


def _isotropic(n):
    """E with <E, u^n> = (u.u)^{n/2}: the coefficient of u^alpha in (x^2 + y^2 + z^2)^{n/2},
    divided by mu_alpha (components store full-tensor entries)."""
    out = []
    for al in sym.multi_indices(n, 3):
        if any(x % 2 for x in al):
            out.append(0.0)
            continue
        h = [x // 2 for x in al]
        coef = math.factorial(n // 2) // (math.factorial(h[0]) * math.factorial(h[1]) * math.factorial(h[2]))
        out.append(coef / sym.multinomial(al))
    return np.array(out)


def _far_starts(a, b, c):
    """Fixed starts where <C, s^n> stays far below both maxima (near c)."""
    return np.stack([_tilt(c, a, 10.0), _tilt(c, b, 10.0), _tilt(c, a + b, 15.0), c])


def test_learned_path_each_branch_against_closed_forms():
    from oracle import ttm
    n = 6
    C, a, b, c = _two_maxima(n)
    cn = np.sqrt(5.0)
    assert sym.frobenius(C, n, 3) == pytest.approx(cn)
    p = mlp.init_params(np.random.default_rng(0), 28)
    far = _far_starts(a, b, c)
    near_a = np.vstack([far, a])

    def run(u0, starts, kappa, **kw):
        return mlp.orient_learned(C, n, p, starts, kappa, u0=u0, **kw)

    # accepted: the search from near a reaches the global maximum, nothing flips
    lam, u, fell = run(_tilt(a, b + c, 8.0), far, 0.5)
    assert not fell and lam == pytest.approx(2.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6
    # accepted at the lower maximum: nothing catches it (no fixed start beats 1)
    lam, u, fell = run(_tilt(b, a + c, 8.0), far, 0.1)
    assert not fell and lam == pytest.approx(1.0, rel=1e-12) and ttm.angle_deg(u, b) < 1e-6
    # lambda / ||C|| < kappa: the multistart runs; the larger answer wins, here the learned one
    lam, u, fell = run(_tilt(a, b + c, 8.0), np.vstack([far, _tilt(b, c, 3.0)]), 0.95)
    assert fell and lam == pytest.approx(2.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6
    # ... and here the multistart's (the learned search sits at b, lambda 1 / sqrt 5 < 0.5)
    lam, u, fell = run(_tilt(b, a + c, 8.0), np.vstack([far, _tilt(a, c, 3.0)]), 0.5)
    assert fell and lam == pytest.approx(2.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6
    # a fixed start beats the learned lambda: <C, a^n> = 2 > 1, so the fallback runs
    lam, u, fell, info = run(_tilt(b, a + c, 8.0), near_a, 0.1, detail=True)
    assert fell and lam == pytest.approx(2.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6
    assert info["beat_gap"] == pytest.approx(cn * (2.0 - 1.0) / cn, rel=1e-9)
    # converged by a loose stopping rule far from the maximum: not certified.
    # C2 = a^n + 2 E, with <E, u^n> = |u|^n, has <C2, u^n> = (a.u)^n + 2 on the
    # sphere: its maximum 3 sits at +-a, and SS-HOPM moves slowly (the radial
    # part of E); one update from 30 degrees away meets tol = 1 with the
    # tangent Hessian not negative definite there, so the fallback runs
    C2 = sym.monomials(a, n) + 2.0 * _isotropic(n)
    lam, u, fell, info = mlp.orient_learned(C2, n, p, near_a, 0.1, u0=_tilt(a, b, 30.0), detail=True,
                                            newton_first=0, tol=1.0, polish=0)
    assert info["converged"] and info["cert_step"] > 1e-2
    assert fell and lam == pytest.approx(3.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6
    # not converged: no Newton step and one SS-HOPM update from far away
    lam, u, fell, info = run(_tilt(c, a, 40.0), near_a, 0.1, detail=True, newton_first=0, max_iter=1)
    assert fell and not info["converged"]
    assert lam == pytest.approx(2.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6


def test_learned_path_zero_tensor_rank_one_and_no_direction():
    from oracle import ttm
    n = 6
    rng = np.random.default_rng(4)
    p = mlp.init_params(rng, 28)
    st = rng.standard_normal((16, 3))
    st /= np.linalg.norm(st, axis=1, keepdims=True)
    lam, u, fell = mlp.orient_learned(np.zeros(28), n, p, st, 0.3)
    assert lam == 0.0 and np.all(u == 0) and not fell
    # rank one: the maximum lam0 at +-v is reached from a start in its basin
    for _ in range(4):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        lam0 = rng.uniform(0.5, 2.0)
        lam, u, fell = mlp.orient_learned(lam0 * sym.monomials(v, n), n, p, st, 0.3,
                                          u0=_tilt(v, rng.standard_normal(3), 20.0))
        assert not fell and lam == pytest.approx(lam0, rel=1e-12) and ttm.angle_deg(u, v) < 1e-6
    # a network with all-zero parameters gives y = 0: no direction, forced fallback,
    # and the answer is the multistart's
    z = {k: np.zeros_like(val) for k, val in p.items()}
    C, a, b, c = _two_maxima(n)
    lam, u, fell = mlp.orient_learned(C, n, z, np.vstack([_far_starts(a, b, c), _tilt(a, c, 5.0)]), -1.0)
    assert fell and lam == pytest.approx(2.0, rel=1e-12) and ttm.angle_deg(u, a) < 1e-6


def test_quaternion_learned_path_rank_one_zero_network_and_layout():
    """The learned path of the quaternion form (d' = 4, degree 4, K = 35, the
    48-input network, no Newton-first steps): on rank-one tensors lam0 q^n the
    answer is (lam0, +-q) with w >= 0 and no fallback, wherever the network
    points (SS-HOPM reaches +-q from any start with u.q != 0, and the value
    lam0 (s.q)^n of every fixed start lies below lam0); a network with zero
    parameters forces the fallback, whose answer is the multistart's; the
    master layout keeps 48 rows of W1 and unpads to the same dict."""
    from oracle import ttm
    n, K, d = 4, 35, 4
    rng = np.random.default_rng(6)
    p = mlp.init_params(rng, K, d_out=d)
    flat = mlp.pad_params(p, K, d)
    assert mlp.padded_inputs(K) == 48 and flat.size == 48 * 64 + 64 + 4096 + 64 + 64 * 16 + 16
    q2 = mlp.unpad_params(flat, K, d)
    assert all(np.array_equal(q2[k], p[k]) for k in p)
    st = rng.standard_normal((32, d))
    st /= np.linalg.norm(st, axis=1, keepdims=True)
    for _ in range(4):
        q = rng.standard_normal(d)
        q /= np.linalg.norm(q)
        lam0 = rng.uniform(0.5, 2.0)
        lam, u, fell = mlp.orient_learned(lam0 * sym.monomials(q, n), n, p, st, 0.3, newton_first=0)
        assert not fell and lam == pytest.approx(lam0, rel=1e-10)
        assert ttm.quat_angle_deg(u, q) < 1e-5 and u[0] >= 0
    z = {k: np.zeros_like(val) for k, val in p.items()}
    C = rng.standard_normal(K)
    lam, u, fell = mlp.orient_learned(C, n, z, st, -1.0, newton_first=0)
    lam_m, u_m, *_ = ttm.orient_multistart(C, n, st)
    assert fell and lam == pytest.approx(lam_m, rel=1e-12) and ttm.quat_angle_deg(u, u_m) < 1e-6
