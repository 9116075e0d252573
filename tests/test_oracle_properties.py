"""Property tests of the oracle on random inputs (hypothesis): identities of
the symmetric-tensor algebra that the tensor template and the tensor field
live in (Sec. 3, Eq. tt; components alpha with multinomial weights), and the
defining property of the greedy Find Peaks result (Sec. 3.4).  Each identity
is checked against a brute-force restatement (full d^n tensors, an explicit
greedy scan), not against the function's own formula."""
import numpy as np
import pytest

pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from oracle import sym, ttm as orc  # noqa: E402

seeds = st.integers(0, 2 ** 31 - 1)


def unit(rng, d):
    u = rng.standard_normal(d)
    return u / np.linalg.norm(u)


def orthogonal(rng, d):
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    return q * np.sign(np.diag(r))


def full_contraction(F, u):
    out = F
    for _ in range(F.ndim):
        out = out @ u
    return float(out)


@settings(max_examples=40, deadline=None)
@given(n=st.sampled_from([2, 4, 6]), d=st.sampled_from([3, 4]), seed=seeds)
def test_inner_power_is_the_full_contraction(n, d, seed):
    """<C, u^n> over the K independent components equals the contraction of the
    full symmetric d^n tensor with n copies of u."""
    if d == 4 and n == 6:
        n = 4   # 4^6 entries: keep the brute force small
    rng = np.random.default_rng(seed)
    C = rng.standard_normal(sym.n_components(n, d))
    u = unit(rng, d)
    F = sym.to_full(C, n, d)
    assert np.isclose(float(sym.inner_power(C, u, n)), full_contraction(F, u), rtol=1e-10, atol=1e-10)


@settings(max_examples=40, deadline=None)
@given(n=st.sampled_from([2, 4]), d=st.sampled_from([3, 4]), seed=seeds)
def test_gradient_contraction_is_the_full_one(n, d, seed):
    """g = C u^{n-1} equals the full tensor contracted with n - 1 copies of u,
    and g . u = <C, u^n>."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal(sym.n_components(n, d))
    u = unit(rng, d)
    F = sym.to_full(C, n, d)
    g_full = F
    for _ in range(n - 1):
        g_full = g_full @ u
    g = sym.contract_n_minus_1(C, u, n)
    assert np.allclose(g, g_full, rtol=1e-10, atol=1e-10)
    assert np.isclose(float(g @ u), float(sym.inner_power(C, u, n)), rtol=1e-10, atol=1e-10)


@settings(max_examples=30, deadline=None)
@given(n=st.sampled_from([2, 4, 6]), seed=seeds)
def test_rotation_moves_the_function_and_keeps_the_norm(n, seed):
    """For an orthogonal G: <G.C, (G u)^n> = <C, u^n> (the form follows the
    rotation) and ||G.C||_F = ||C||_F, with G.C formed on the full tensor."""
    rng = np.random.default_rng(seed)
    d = 3
    C = rng.standard_normal(sym.n_components(n, d))
    G = orthogonal(rng, d)
    u = unit(rng, d)
    CG = sym.rotate(C, G, n)
    assert np.isclose(float(sym.inner_power(CG, G @ u, n)), float(sym.inner_power(C, u, n)),
                      rtol=1e-9, atol=1e-9)
    FG = sym.to_full(CG, n, d)
    assert np.isclose(float(sym.frobenius(CG, n, d)), float(np.sqrt(np.sum(FG * FG))), rtol=1e-10)
    assert np.isclose(float(sym.frobenius(CG, n, d)), float(sym.frobenius(C, n, d)), rtol=1e-9)


@settings(max_examples=40, deadline=None)
@given(seed=seeds, shape=st.tuples(st.integers(3, 9), st.integers(3, 9), st.integers(3, 9)),
       levels=st.integers(2, 6), top_p=st.integers(1, 30),
       dist=st.sampled_from([0.0, 1.0, 1.5, 2.0, 3.0]))
def test_find_peaks_is_the_greedy_scan(seed, shape, levels, top_p, dist):
    """Find Peaks on maps with many ties: peak k holds the largest score among
    the valid voxels other than peaks 0..k-1 and at distance >= min_dist from
    them (smallest linear index on ties), and the list stops only at P peaks
    or when no such voxel is left."""
    rng = np.random.default_rng(seed)
    m = rng.integers(0, levels, shape).astype(np.float64)
    lo = tuple(int(rng.integers(0, s // 2)) for s in shape)
    hi = tuple(int(rng.integers(l, s)) for l, s in zip(lo, shape))
    pk, pv = orc.find_peaks(m, lo, hi, top_p, dist)
    cand = [(z, y, x) for z in range(lo[0], hi[0] + 1) for y in range(lo[1], hi[1] + 1)
            for x in range(lo[2], hi[2] + 1)]
    kept = []

    def free_voxels():
        # not taken yet, and min_dist or farther from every kept peak (a
        # distance of 0 excludes only the peaks themselves)
        return [c for c in cand if c not in kept and
                all(np.sum((np.array(c) - np.array(q)) ** 2) >= dist * dist for q in kept)]
    for k in range(len(pk)):
        free = free_voxels()
        best = max(m[c] for c in free)
        first = min((c for c in free if m[c] == best), key=lambda c: np.ravel_multi_index(c, shape))
        assert tuple(pk[k]) == first and pv[k] == best
        kept.append(first)
    if len(pk) < top_p:
        assert not free_voxels()
