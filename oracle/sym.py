"""Symmetric-tensor algebra (FP64).  TEST INFRASTRUCTURE ONLY (see oracle/__init__).

A degree-n symmetric tensor over R^d is stored by its independent components,
one per multi-index alpha in N^d with |alpha| = n (Sec. 3, Alg. 1: "indices of
the independent components"; their count is binom(n+d-1, n), Sec. 3 after
Alg. 2).  Component alpha holds the full-tensor entry shared by all index
tuples with those counts, so "component i of q^{(.)n}" is the monomial
q^alpha (Alg. 1).  Inner products and the Frobenius norm therefore carry the
multinomial weight mu_alpha = n!/prod(alpha_i!), the number of index tuples
per component.

Order of components: graded-lex, i.e. descending alpha_0, then descending
alpha_1, and so on.

Pins (tests/test_oracle_sym.py): the full-tensor expansion is checked against
brute-force sums over all d^n index tuples; sphere moments against the closed
form of Gaussian integrals; contractions against finite differences.
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def multi_indices(n: int, d: int) -> tuple:
    """All alpha in N^d with |alpha| = n, graded-lex (descending leading counts)."""
    if d == 1:
        return ((n,),)
    out = []
    for a0 in range(n, -1, -1):
        for rest in multi_indices(n - a0, d - 1):
            out.append((a0,) + rest)
    return tuple(out)


def n_components(n: int, d: int) -> int:
    return math.comb(n + d - 1, n)


def multinomial(alpha) -> int:
    n = sum(alpha)
    out = math.factorial(n)
    for a in alpha:
        out //= math.factorial(a)
    return out


def weights(n: int, d: int) -> np.ndarray:
    return np.array([multinomial(a) for a in multi_indices(n, d)], dtype=np.float64)


def monomials(v: np.ndarray, n: int) -> np.ndarray:
    """v^alpha for every alpha (graded-lex); v has shape (..., d) -> (..., K)."""
    v = np.asarray(v, dtype=np.float64)
    d = v.shape[-1]
    al = np.array(multi_indices(n, d))                    # (K, d)
    return np.prod(v[..., None, :] ** al, axis=-1)


def index_of(n: int, d: int) -> dict:
    return {a: i for i, a in enumerate(multi_indices(n, d))}


def inner_power(C: np.ndarray, u: np.ndarray, n: int) -> np.ndarray:
    """<C, u^{(x)n}> = sum_alpha mu_alpha C_alpha u^alpha.  C: (K, ...), u: (d,)."""
    d = len(u)
    w = weights(n, d) * monomials(np.asarray(u), n)
    return np.tensordot(w, C, axes=(0, 0))


@lru_cache(maxsize=None)
def _raise_table(n: int, d: int):
    """For every |beta| = n-1: mu_beta and the component index of beta + e_i, i < d."""
    idx = index_of(n, d)
    betas = multi_indices(n - 1, d)
    mu = np.array([multinomial(b) for b in betas], dtype=np.float64)
    tab = np.empty((len(betas), d), dtype=np.int64)
    for k, beta in enumerate(betas):
        for i in range(d):
            a = list(beta)
            a[i] += 1
            tab[k, i] = idx[tuple(a)]
    return mu, tab


def contract_n_minus_1(C: np.ndarray, u: np.ndarray, n: int) -> np.ndarray:
    """(C u^{n-1})_i = sum_{|beta|=n-1} mu_beta C_{beta+e_i} u^beta, shape (d,).

    This is one n-th of the gradient of <C, u^{(x)n}> with respect to u.
    """
    u = np.asarray(u, dtype=np.float64)
    d = len(u)
    mu, tab = _raise_table(n, d)
    wb = mu * monomials(u, n - 1)                         # (K_{n-1},)
    return wb @ np.asarray(C, dtype=np.float64)[tab]      # (d,)


def contract_n_minus_2(C: np.ndarray, u: np.ndarray, n: int) -> np.ndarray:
    """(C u^{n-2})_{ij} = sum_{|beta|=n-2} mu_beta C_{beta+e_i+e_j} u^beta, a d x d matrix.

    It is 1/(n(n-1)) of the Hessian of <C, u^{(x)n}>.
    """
    u = np.asarray(u, dtype=np.float64)
    d = len(u)
    idx = index_of(n, d)
    H = np.zeros((d, d))
    for beta in multi_indices(n - 2, d):
        mb = multinomial(beta) * np.prod(u ** np.array(beta))
        for i in range(d):
            for j in range(d):
                a = list(beta)
                a[i] += 1
                a[j] += 1
                H[i, j] += mb * C[idx[tuple(a)]]
    return H


def frobenius(C: np.ndarray, n: int, d: int) -> np.ndarray:
    """||C||_F over the full tensor: sqrt(sum_alpha mu_alpha C_alpha^2).  C: (K, ...)."""
    w = weights(n, d)
    return np.sqrt(np.tensordot(w, np.asarray(C, dtype=np.float64) ** 2, axes=(0, 0)))


def counts_of(tup, d: int) -> tuple:
    c = [0] * d
    for i in tup:
        c[i] += 1
    return tuple(c)


def to_full(C: np.ndarray, n: int, d: int) -> np.ndarray:
    """Expand independent components (K,) into the full d^n array."""
    idx = index_of(n, d)
    full = np.empty((d,) * n)
    for tup in itertools.product(range(d), repeat=n):
        full[tup] = C[idx[counts_of(tup, d)]]
    return full


def from_full(F: np.ndarray, n: int, d: int) -> np.ndarray:
    """Read the independent components off a symmetric full tensor."""
    out = np.empty(n_components(n, d))
    for i, a in enumerate(multi_indices(n, d)):
        tup = tuple(j for j in range(d) for _ in range(a[j]))
        out[i] = F[tup]
    return out


def rotate_full(F: np.ndarray, G: np.ndarray) -> np.ndarray:
    """(G.F)_{i1..in} = sum_j G_{i1 j1} ... G_{in jn} F_{j1..jn}."""
    out = F
    n = F.ndim
    for ax in range(n):
        out = np.moveaxis(np.tensordot(G, out, axes=(1, ax)), 0, ax)
    return out


def rotate(C: np.ndarray, G: np.ndarray, n: int) -> np.ndarray:
    d = G.shape[0]
    return from_full(rotate_full(to_full(C, n, d), G), n, d)


def double_factorial(k: int) -> int:
    if k <= 0:
        return 1
    out = 1
    while k > 1:
        out *= k
        k -= 2
    return out


def sphere_moment(alpha) -> float:
    """E[prod x_i^alpha_i] for x uniform on the unit sphere S^{d-1} in R^d.

    Zero unless every alpha_i is even; otherwise
    prod (alpha_i - 1)!! / (d (d+2) ... (d+n-2)).
    """
    d = len(alpha)
    n = sum(alpha)
    if any(a % 2 for a in alpha):
        return 0.0
    num = 1
    for a in alpha:
        num *= double_factorial(a - 1)
    den = 1
    for k in range(0, n, 2):
        den *= d + k
    return num / den


def unfolding(C: np.ndarray, n: int, d: int) -> np.ndarray:
    """Square matrix unfolding d^{n/2} x d^{n/2} of the full tensor (n even)."""
    F = to_full(C, n, d)
    m = d ** (n // 2)
    return F.reshape(m, m)


def unfolding_symmetric_block(C: np.ndarray, n: int, d: int) -> np.ndarray:
    """The unfolding restricted to symmetric (n/2)-tensors, in an orthonormal basis.

    Every row of the unfolding depends only on the multiset of its row index,
    so the unfolding vanishes off the symmetric subspace; there it is the
    K_{n/2} x K_{n/2} matrix B[beta, gamma] = sqrt(mu_beta mu_gamma) C_{beta+gamma}.
    Its eigenvalues are the non-zero eigenvalues of the unfolding.
    """
    half = multi_indices(n // 2, d)
    idx = index_of(n, d)
    B = np.empty((len(half), len(half)))
    for i, b in enumerate(half):
        for j, c in enumerate(half):
            B[i, j] = math.sqrt(multinomial(b) * multinomial(c)) * C[idx[tuple(np.add(b, c))]]
    return B
