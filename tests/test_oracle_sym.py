"""Pins of the oracle's symmetric-tensor algebra against brute force and closed forms."""
import itertools
import math

import numpy as np
import pytest

from oracle import sym


@pytest.mark.parametrize("n,d", [(2, 3), (4, 3), (6, 3), (4, 4), (6, 4), (0, 3)])
def test_component_count_and_order(n, d):
    al = sym.multi_indices(n, d)
    assert len(al) == math.comb(n + d - 1, n) == sym.n_components(n, d)
    assert len(set(al)) == len(al)
    assert all(sum(a) == n and min(a) >= 0 for a in al)
    # graded-lex: descending first count, then second, ...
    assert list(al) == sorted(al, reverse=True)


def test_component_counts_paper():
    # binom(n + d' - 1, n) = 35 for n = 4, d' = 4 (Sec. 3, after Alg. 2)
    assert sym.n_components(4, 4) == 35
    assert sym.n_components(4, 3) == 15 and sym.n_components(6, 3) == 28


def test_multinomial_counts_tuples():
    for n, d in [(4, 3), (6, 3), (4, 4)]:
        counts = {}
        for tup in itertools.product(range(d), repeat=n):
            c = sym.counts_of(tup, d)
            counts[c] = counts.get(c, 0) + 1
        for a in sym.multi_indices(n, d):
            assert counts[a] == sym.multinomial(a)


@pytest.mark.parametrize("n,d", [(4, 3), (6, 3), (4, 4)])
def test_full_tensor_brute_force(n, d):
    rng = np.random.default_rng(n * 10 + d)
    C = rng.standard_normal(sym.n_components(n, d))
    F = sym.to_full(C, n, d)
    # symmetric under every index permutation
    for perm in list(itertools.permutations(range(n)))[:20]:
        assert np.array_equal(F, np.transpose(F, perm))
    assert np.allclose(sym.from_full(F, n, d), C)
    # Frobenius norm = sqrt(sum over all d^n entries)
    assert np.isclose(sym.frobenius(C, n, d), np.sqrt(np.sum(F * F)), rtol=1e-13)
    # <C, u^n> = full contraction
    u = rng.standard_normal(d)
    full = F
    for _ in range(n):
        full = full @ u
    assert np.isclose(sym.inner_power(C, u, n), full, rtol=1e-12)
    # (C u^{n-1})_i = full contraction on n-1 indices
    g = F
    for _ in range(n - 1):
        g = g @ u
    assert np.allclose(sym.contract_n_minus_1(C, u, n), g, rtol=1e-12)


@pytest.mark.parametrize("n,d", [(4, 3), (6, 3), (4, 4)])
def test_contraction_is_gradient_over_n(n, d):
    rng = np.random.default_rng(3)
    C = rng.standard_normal(sym.n_components(n, d))
    u = rng.standard_normal(d)
    h = 1e-6
    grad = np.array([(sym.inner_power(C, u + h * e, n) - sym.inner_power(C, u - h * e, n)) / (2 * h)
                     for e in np.eye(d)])
    assert np.allclose(grad / n, sym.contract_n_minus_1(C, u, n), rtol=1e-6, atol=1e-8)


def test_rank_one_monomials():
    # v^{(x)n} has components v^alpha and Frobenius norm |v|^n
    rng = np.random.default_rng(4)
    for n, d in [(4, 3), (6, 3), (4, 4)]:
        v = rng.standard_normal(d)
        C = sym.monomials(v, n)
        F = sym.to_full(C, n, d)
        outer = v
        for _ in range(n - 1):
            outer = np.multiply.outer(outer, v)
        assert np.allclose(F, outer)
        assert np.isclose(sym.frobenius(C, n, d), np.linalg.norm(v) ** n)


def test_sphere_moments_textbook():
    # E[x^4] = 1/5, E[x^2 y^2] = 1/15, E[x^6] = 1/7 on S^2; E[x^2] = 1/d
    assert sym.sphere_moment((4, 0, 0)) == pytest.approx(1 / 5)
    assert sym.sphere_moment((2, 2, 0)) == pytest.approx(1 / 15)
    assert sym.sphere_moment((6, 0, 0)) == pytest.approx(1 / 7)
    assert sym.sphere_moment((2, 0, 0, 0)) == pytest.approx(1 / 4)
    assert sym.sphere_moment((3, 1, 0)) == 0.0


def test_sphere_moments_quadrature():
    # independent check: product Gauss-Legendre x trapezoid quadrature on S^2
    nt, nphi = 64, 128
    xs, ws = np.polynomial.legendre.leggauss(nt)        # cos(theta)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xs, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    pts = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1)
    wt = (ws[:, None] * np.ones(nphi)[None, :]) * (2 * np.pi / nphi) / (4 * np.pi)
    for a in sym.multi_indices(6, 3):
        val = np.sum(wt * np.prod(pts ** np.array(a), axis=-1))
        assert val == pytest.approx(sym.sphere_moment(a), abs=1e-12)


def test_rotation_invariance_of_frobenius():
    rng = np.random.default_rng(5)
    for n, d in [(4, 3), (6, 3), (4, 4)]:
        C = rng.standard_normal(sym.n_components(n, d))
        G, _ = np.linalg.qr(rng.standard_normal((d, d)))
        Cr = sym.rotate(C, G, n)
        assert np.isclose(sym.frobenius(Cr, n, d), sym.frobenius(C, n, d), rtol=1e-12)
        u = rng.standard_normal(d)
        # <G.C, (G u)^n> = <C, u^n>
        assert np.isclose(sym.inner_power(Cr, G @ u, n), sym.inner_power(C, u, n), rtol=1e-11)


@pytest.mark.parametrize("n,d", [(4, 3), (6, 3), (4, 4)])
def test_unfolding_symmetric_block(n, d):
    rng = np.random.default_rng(6)
    C = rng.standard_normal(sym.n_components(n, d))
    U = sym.unfolding(C, n, d)
    B = sym.unfolding_symmetric_block(C, n, d)
    ev_u = np.sort(np.linalg.eigvalsh(U))
    ev_b = np.sort(np.linalg.eigvalsh(B))
    nz = ev_u[np.abs(ev_u) > 1e-9]
    assert len(nz) <= len(ev_b)
    assert np.allclose(np.sort(nz), np.sort(ev_b[np.abs(ev_b) > 1e-9]), atol=1e-10)
    assert np.isclose(min(0.0, ev_u.min()), min(0.0, ev_b.min()), atol=1e-10)


@pytest.mark.parametrize("n,d", [(4, 3), (6, 3), (4, 4)])
def test_second_contraction_is_jacobian(n, d):
    rng = np.random.default_rng(7)
    C = rng.standard_normal(sym.n_components(n, d))
    u = rng.standard_normal(d)
    H = sym.contract_n_minus_2(C, u, n)
    h = 1e-6
    J = np.stack([(sym.contract_n_minus_1(C, u + h * e, n) - sym.contract_n_minus_1(C, u - h * e, n)) / (2 * h)
                  for e in np.eye(d)], axis=1)
    assert np.allclose(J, (n - 1) * H, rtol=1e-6, atol=1e-8)
    assert np.allclose(H, H.T)
