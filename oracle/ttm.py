"""Tensorial template matching, FP64 reference.  TEST INFRASTRUCTURE ONLY (see oracle/__init__).

Everything here is the plain definition written out, in the paper's order:

* filter h with 1D z-transform 1 + a(z + z^-1 - 2), a = 1/5, separable
  (Sec. 2, after Eq. norm_f)                                   -> prefilter_*
* binary ball mask m, M = sum m (Sec. 2; soft edge not used)   -> ball_mask
* template zero-normalisation t' (Eq. norm_t)                  -> normalize_template
* tensor template T_alpha = (1/N_q) sum_q v_q^alpha t'_q (Eq. tt, Alg. 1)
                                                               -> tensor_template
* local normalisation w(x) (Eq. norm_f)                        -> local_normalization
* tensor field C_alpha = w (g * T_alpha), a correlation (Eq. tcc, Alg. 2,
  Eq. correlation), by direct spatial sums                     -> tensor_field
* Frobenius score ||C||_F (Sec. 3.2)                           -> score
* SS-HOPM dominant eigenpair from given starts (Sec. 3.1)      -> sshopm, converge,
                                                                  orient_multistart
* Find Peaks: P highest scores at least two mask radii apart (Sec. 3.4)
                                                               -> find_peaks
* position refinement TTM-ref (Sec. 3.3, Alg. 3)              -> refine_positions
* rotation-sampled TM c(x, R) = w (f * t'_R) (Eq. lncc)        -> brute_force_tm, lncc_at

Readings of points the paper leaves open:
* the image operator S reduces to h* on the image; the mask acts through t'
  and w; correlation outputs exist only on the valid region, where the whole
  template box lies inside the volume, and are 0 elsewhere;
* g = h*f replicates the border voxel on the volume, t is zero-padded;
* Alg. 1 rotates t', which already contains S, so no second filtering;
* template centre c = L//2 per axis, mask m(p) = [|p - c|^2 <= r^2];
* d' = 3 axis form: v_q = R(q) a for a fixed template axis a (default z);
  d' = 4: v_q = q itself, the paper's quaternion form;
* w = 0 where var <= eps_w * M * mean(g^2 over the volume), eps_w = 1e-6;
* SS-HOPM maximises the signed value, on the tensor divided by its Frobenius
  norm; its shift is alpha = max(0, -lambda_min(U)) with U the square matrix
  unfolding (the paper's rule, Sec. 3.1).  The paper states no stopping rule;
  the oracle computes the converged maximum of each start's basin: SS-HOPM
  until |delta lambda| <= 1e-13 or 10^4 updates, then Newton's method on the
  sphere until lambda changes by <= 1e-15 (the same fixed point, reached
  quadratically); best start by largest lambda, lowest index on ties; sign
  canonicalised so the last non-zero coordinate is positive (d' = 3) or the
  scalar part of the quaternion is (d' = 4).

Parity status: every function here is pinned by tests/test_oracle_*.py
(closed forms, invariants, brute force, textbook routines); the absolute
values on the synthetic workloads are not printed in the paper.
"""
from __future__ import annotations

import math

import numpy as np

from . import sym
from .rotations import quat_to_matrix, rotate_template

# ----------------------------------------------------------------------------
# filter, mask, template normalisation
# ----------------------------------------------------------------------------


def filter_taps(a: float = 0.2) -> np.ndarray:
    """Impulse response of 1 + a(z + z^-1 - 2): [a, 1 - 2a, a]."""
    return np.array([a, 1.0 - 2.0 * a, a])


def _filter_axis(x: np.ndarray, axis: int, a: float, mode: str) -> np.ndarray:
    taps = filter_taps(a)
    pad = [(0, 0)] * x.ndim
    pad[axis] = (1, 1)
    xp = np.pad(x, pad, mode=mode)
    n = x.shape[axis]
    lo = np.take(xp, np.arange(0, n), axis=axis)
    mid = np.take(xp, np.arange(1, n + 1), axis=axis)
    hi = np.take(xp, np.arange(2, n + 2), axis=axis)
    return taps[0] * lo + taps[1] * mid + taps[2] * hi


def prefilter_volume(f: np.ndarray, a: float = 0.2) -> np.ndarray:
    """g = h * f, separable over z, y, x, border voxels replicated."""
    g = np.asarray(f, dtype=np.float64)
    for ax in range(3):
        g = _filter_axis(g, ax, a, "edge")
    return g


def prefilter_box(f: np.ndarray, lo, hi, a: float = 0.2) -> np.ndarray:
    """g = h * f restricted to the box [lo, hi) (z, y, x) of a larger volume.

    Same values as prefilter_volume(f)[box]; only reads f around the box.
    """
    sl = []
    pad = []
    for ax in range(3):
        a0, a1 = lo[ax] - 1, hi[ax] + 1
        c0, c1 = max(a0, 0), min(a1, f.shape[ax])
        sl.append(slice(c0, c1))
        pad.append((c0 - a0, a1 - c1))
    sub = np.pad(np.asarray(f[tuple(sl)], dtype=np.float64), pad, mode="edge")
    g = sub
    taps = filter_taps(a)
    for ax in range(3):
        n = g.shape[ax] - 2
        g = (taps[0] * np.take(g, np.arange(0, n), axis=ax)
             + taps[1] * np.take(g, np.arange(1, n + 1), axis=ax)
             + taps[2] * np.take(g, np.arange(2, n + 2), axis=ax))
        # the margin of the other axes stays until they are filtered
    return g


def prefilter_template(t: np.ndarray, a: float = 0.2) -> np.ndarray:
    """h * t with zero padding outside the template box."""
    g = np.asarray(t, dtype=np.float64)
    for ax in range(3):
        g = _filter_axis(g, ax, a, "constant")
    return g


def ball_mask(L: int, r: float) -> np.ndarray:
    """m(p) = 1 if |p - c| <= r else 0, c = L//2 on every axis."""
    idx = np.arange(L) - L // 2
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    return ((xx * xx + yy * yy + zz * zz) <= r * r).astype(np.float64)


def normalize_template(t: np.ndarray, r: float, a: float = 0.2) -> np.ndarray:
    """t' = m (S(t) - mu) / sqrt(<S(t)^2, 1> - <S(t), 1>^2 / M)   (Eq. norm_t).

    S(t) = m (h * t); mu = <S(t), m> / M.
    """
    m = ball_mask(t.shape[0], r)
    M = m.sum()
    st = m * prefilter_template(t, a)
    mu = np.sum(st * m) / M
    sig = math.sqrt(np.sum(st * st) - np.sum(st) ** 2 / M)
    return m * (st - mu) / sig


# ----------------------------------------------------------------------------
# tensor template (Alg. 1)
# ----------------------------------------------------------------------------


def direction_of(q, dprime: int, axis=(0.0, 0.0, 1.0)) -> np.ndarray:
    """The vector whose n-th power stands for rotation q: R(q) a (d'=3) or q (d'=4)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    if dprime == 4:
        return q
    return quat_to_matrix(q) @ np.asarray(axis, dtype=np.float64)


def tensor_template(tn: np.ndarray, quats: np.ndarray, n: int, dprime: int = 3,
                    axis=(0.0, 0.0, 1.0)) -> np.ndarray:
    """T_alpha(p) = (1/N_q) sum_q v_q^alpha t'_q(p), shape (K, L, L, L).

    For each q: rotate t' (trilinear pull-back), then add the monomial-weighted
    copy to every component (Alg. 1), with equal quadrature weights 1/N_q.
    """
    L = tn.shape[0]
    K = sym.n_components(n, dprime)
    T = np.zeros((K, L, L, L))
    for q in quats:
        tq = rotate_template(tn, quat_to_matrix(q))
        k = sym.monomials(direction_of(q, dprime, axis), n)
        T += k[:, None, None, None] * tq[None]
    return T / len(quats)


def wedge_keep(P: int, half_angle_deg: float) -> np.ndarray:
    """Missing-wedge filter on the half spectrum of a real P^3 box (numpy.fft.rfftn
    layout [kz][ky][kx], kx halved): 1 where a Fourier coefficient is kept, 0 where
    |k_z| > tan(angle) |k_x| (tilt axis y, beam z, as the tomogram's wedge); the
    DC coefficient is kept."""
    kz = np.fft.fftfreq(P)[:, None, None]
    kx = np.fft.rfftfreq(P)[None, None, :]
    drop = np.abs(kz) > np.tan(np.radians(half_angle_deg)) * np.abs(kx)
    keep = np.broadcast_to(~drop, (P, P, P // 2 + 1)).astype(np.float64).copy()
    keep[0, 0, 0] = 1.0
    return keep


def mask_normalize(v: np.ndarray, m: np.ndarray) -> np.ndarray:
    """m (v - mu) / sigma over the mask m (Eq. norm_t without the prefilter):
    mu = <v, m> / M, sigma^2 = <v^2, m> - <v, m>^2 / M."""
    v = np.asarray(v, dtype=np.float64)
    M = float(m.sum())
    s1 = float((v * m).sum())
    s2 = float((v * v * m).sum())
    return m * (v - s1 / M) / np.sqrt(s2 - s1 * s1 / M)


def tensor_template_wedge(tn: np.ndarray, quats: np.ndarray, n: int, r: float,
                          half_angle_deg: float | None, P: int, dprime: int = 3,
                          axis=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Wedge-aware tensor template (a reading of Eq. tt for tomograms with a
    missing wedge): T_alpha = (1/N_q) sum_q v_q^alpha N_m(W t'_q), where t'_q is
    t' rotated by R(q) as in tensor_template, W the tomogram's missing-wedge
    filter applied on the template box zero-padded to P^3 (periodic FFT; the
    wedge lies in the tomogram's frame, so it acts after the rotation), and N_m
    the renormalisation over the mask (mask_normalize), so that every rotated,
    filtered template has zero mean and unit norm on the mask.  With
    half_angle_deg None, W is the identity."""
    L = tn.shape[0]
    m = ball_mask(L, r)
    keep = None if half_angle_deg is None else wedge_keep(P, half_angle_deg)
    K = sym.n_components(n, dprime)
    T = np.zeros((K, L, L, L))
    for q in quats:
        tq = rotate_template(tn, quat_to_matrix(q))
        if keep is not None:
            box = np.zeros((P, P, P))
            box[:L, :L, :L] = tq
            tq = np.fft.irfftn(np.fft.rfftn(box) * keep, s=(P, P, P), axes=(0, 1, 2))[:L, :L, :L]
        tq = mask_normalize(tq, m)
        k = sym.monomials(direction_of(q, dprime, axis), n)
        T += k[:, None, None, None] * tq[None]
    return T / len(quats)


# ----------------------------------------------------------------------------
# valid region, local normalisation, tensor field
# ----------------------------------------------------------------------------


def valid_range(D: int, L: int):
    """First and last voxel whose template window [x - c, x - c + L) lies inside [0, D)."""
    c = L // 2
    return c, D - L + c


def _windows(g: np.ndarray, L: int):
    return np.lib.stride_tricks.sliding_window_view(g, (L, L, L))


def correlate_valid(g: np.ndarray, kernels: np.ndarray) -> np.ndarray:
    """out[k, v] = sum_p g[v + p] kernels[k, p] for every v with the window inside g.

    This is (g * t)(x) = sum_p g(x + p - c) t(p) (Eq. correlation) at the valid
    voxel x = v + c.  kernels: (nk, L, L, L) -> (nk, Vz, Vy, Vx).
    """
    L = kernels.shape[-1]
    win = _windows(np.asarray(g, dtype=np.float64), L)
    Vz, Vy, Vx = win.shape[:3]
    km = kernels.reshape(kernels.shape[0], -1).T                      # (L^3, nk)
    out = np.empty((kernels.shape[0], Vz, Vy, Vx))
    rows = max(1, int(2 ** 25 // max(1, Vx * L ** 3)))
    for z in range(Vz):
        for y0 in range(0, Vy, rows):
            y1 = min(Vy, y0 + rows)
            patch = win[z, y0:y1].reshape(-1, L ** 3)
            out[:, z, y0:y1, :] = (patch @ km).T.reshape(-1, y1 - y0, Vx)
    return out


def volume_g2_mean(g: np.ndarray) -> float:
    return float(np.mean(np.asarray(g, dtype=np.float64) ** 2))


def local_variance(g: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """var(x) = <S(tau_x g)^2, 1> - <S(tau_x g), 1>^2 / M on the valid region (Eq. norm_f)."""
    M = mask.sum()
    s1 = correlate_valid(g, mask[None])[0]
    s2 = correlate_valid(np.asarray(g, dtype=np.float64) ** 2, (mask * mask)[None])[0]
    return s2 - s1 * s1 / M


def local_normalization(g: np.ndarray, mask: np.ndarray, eps_w: float = 1e-6,
                        g2_mean: float | None = None) -> np.ndarray:
    """w(x) = 1 / sqrt(var(x)) on the valid region, 0 elsewhere (Eq. norm_f).

    Guard: w = 0 where var <= eps_w * M * mean(g^2) (a flat or constant window).
    Returns a full-size map.
    """
    L = mask.shape[0]
    M = mask.sum()
    if g2_mean is None:
        g2_mean = volume_g2_mean(g)
    var = local_variance(g, mask)
    w_valid = np.where(var > eps_w * M * g2_mean, 1.0 / np.sqrt(np.maximum(var, 1e-300)), 0.0)
    w = np.zeros(g.shape)
    c = L // 2
    Vz, Vy, Vx = var.shape
    w[c:c + Vz, c:c + Vy, c:c + Vx] = w_valid
    return w


def tensor_field(g: np.ndarray, w: np.ndarray, T: np.ndarray) -> np.ndarray:
    """C_alpha(x) = w(x) (g * T_alpha)(x) on the valid region (Eq. tcc, Alg. 2).

    Returns (K, Vz, Vy, Vx) indexed from the first valid voxel.
    """
    L = T.shape[-1]
    c = L // 2
    raw = correlate_valid(g, T)
    Vz, Vy, Vx = raw.shape[1:]
    return raw * w[None, c:c + Vz, c:c + Vy, c:c + Vx]


def patches_at(g_box_source, points, L: int, f=None, a: float = 0.2):
    """Template windows g[x - c : x - c + L] at the given voxels (N, 3) (z, y, x).

    If ``f`` is given, g = h * f is evaluated on each window from f (replicated
    borders) instead of reading a precomputed g.
    """
    c = L // 2
    out = np.empty((len(points), L, L, L))
    for i, (z, y, x) in enumerate(points):
        lo = (z - c, y - c, x - c)
        hi = (z - c + L, y - c + L, x - c + L)
        if f is not None:
            out[i] = prefilter_box(f, lo, hi, a)
        else:
            out[i] = g_box_source[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
    return out


def field_at(patches: np.ndarray, mask: np.ndarray, T: np.ndarray, g2_mean: float,
             eps_w: float = 1e-6):
    """w, C at individual voxels from their template windows (same sums as above)."""
    M = mask.sum()
    P = patches.reshape(len(patches), -1)
    s1 = P @ mask.reshape(-1)
    s2 = (P * P) @ (mask * mask).reshape(-1)
    var = s2 - s1 * s1 / M
    w = np.where(var > eps_w * M * g2_mean, 1.0 / np.sqrt(np.maximum(var, 1e-300)), 0.0)
    C = (P @ T.reshape(T.shape[0], -1).T) * w[:, None]                # (N, K)
    return w, C


# ----------------------------------------------------------------------------
# score and orientation
# ----------------------------------------------------------------------------


def score(C: np.ndarray, n: int, dprime: int = 3) -> np.ndarray:
    """c_hat = ||C||_F = sqrt(sum_alpha mu_alpha C_alpha^2) (Sec. 3.2).  C: (K, ...)."""
    return sym.frobenius(C, n, dprime)


def canonical_sign(u: np.ndarray) -> np.ndarray:
    """u and -u are one answer.  d' = 3 (an axis): the last non-zero coordinate is
    made positive; d' = 4 (a quaternion w, x, y, z): the first (w) is."""
    u = np.array(u, dtype=np.float64)
    order = range(len(u)) if len(u) == 4 else range(len(u) - 1, -1, -1)
    for i in order:
        if u[i] != 0.0:
            return u if u[i] > 0 else -u
    return u


def gradient_many(Cv: np.ndarray, n: int, U: np.ndarray) -> np.ndarray:
    """Rows of C u^{n-1} for every row u of U (S, d) -> (S, d)."""
    mu, tab = sym._raise_table(n, U.shape[1])
    return (mu * sym.monomials(U, n - 1)) @ np.asarray(Cv, dtype=np.float64)[tab]


def sshopm(Cv: np.ndarray, n: int, u0, alpha: float, tol: float, max_iter: int):
    """Shifted symmetric higher-order power method (Kolda & Mayo), maximising.

    u <- (C u^{n-1} + alpha u) / ||.||;  lambda = <C, u^{(x)n}>.
    Stops when |lambda_new - lambda| <= tol or after max_iter updates.
    u0 is one start (d,) or several (S, d), each run on its own (a run that has
    stopped is left as it is while the others go on).
    Returns (lambda, u, iterations, converged), per start when u0 is 2-D.
    """
    U = np.atleast_2d(np.asarray(u0, dtype=np.float64))
    U = U / np.linalg.norm(U, axis=1, keepdims=True)
    S = U.shape[0]
    G = gradient_many(Cv, n, U)
    lam = np.sum(G * U, axis=1)
    its = np.zeros(S, dtype=np.int64)
    conv = np.zeros(S, dtype=bool)
    live = np.ones(S, dtype=bool)
    for it in range(1, max_iter + 1):
        if not live.any():
            break
        V = G[live] + alpha * U[live]
        Un = V / np.linalg.norm(V, axis=1, keepdims=True)
        Gn = gradient_many(Cv, n, Un)
        ln = np.sum(Gn * Un, axis=1)
        idx = np.flatnonzero(live)
        done = np.abs(ln - lam[idx]) <= tol
        U[idx], G[idx], lam[idx], its[idx] = Un, Gn, ln, it
        conv[idx[done]] = True
        live[idx[done]] = False
    if np.ndim(u0) == 1:
        return float(lam[0]), U[0], int(its[0]), bool(conv[0])
    return lam, U, its, conv


def unfolding_shift(Cu: np.ndarray, n: int, d: int) -> float:
    """alpha = max(0, -lambda_min(U)), U the d^{n/2} x d^{n/2} unfolding (Sec. 3.1)."""
    return max(0.0, -float(np.linalg.eigvalsh(sym.unfolding(Cu, n, d)).min()))


def tangent_basis(u: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the plane orthogonal to unit u, as d - 1 columns
    (the last d - 1 columns of the QR factor of [u | I])."""
    u = np.asarray(u, dtype=np.float64)
    d = len(u)
    Q, _ = np.linalg.qr(np.column_stack([u, np.eye(d)]))
    return Q[:, 1:d]


def tangent_hessian(Cu: np.ndarray, n: int, u: np.ndarray, lam: float, E: np.ndarray) -> np.ndarray:
    """Hessian of <C, u^n> / n on the sphere in the tangent basis E:
    (n - 1) E^T (C u^{n-2}) E - lambda I."""
    return (n - 1) * (E.T @ sym.contract_n_minus_2(Cu, u, n) @ E) - lam * np.eye(E.shape[1])


def newton_direction(Cu: np.ndarray, n: int, u: np.ndarray, g: np.ndarray, lam: float):
    """Riemannian Newton direction for max <C, u^n> on the unit sphere at u
    (g = C u^{n-1}, lambda = g.u), or None where the tangent Hessian is not
    negative definite (u is then not near a local maximum)."""
    E = tangent_basis(u)
    Ht = tangent_hessian(Cu, n, u, lam, E)
    if not np.all(np.linalg.eigvalsh(Ht) < 0.0):
        return None
    return E @ (-np.linalg.solve(Ht, E.T @ g))


def newton_finish(Cu: np.ndarray, n: int, u: np.ndarray, max_steps: int = 30):
    """Newton's method on the sphere from a point SS-HOPM has brought near a
    local maximum, until a step changes lambda by at most 1e-15: the fixed point
    that SS-HOPM converges to, reached quadratically instead of linearly.
    A step is taken only where the tangent Hessian is negative definite and
    kept only if lambda does not fall by more than 1e-15.  Returns (lambda, u)."""
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    g = sym.contract_n_minus_1(Cu, u, n)
    lam = float(g @ u)
    for _ in range(max_steps):
        dvec = newton_direction(Cu, n, u, g, lam)
        if dvec is None:
            break
        un = u + dvec
        un = un / np.linalg.norm(un)
        gn = sym.contract_n_minus_1(Cu, un, n)
        ln = float(gn @ un)
        if ln < lam - 1e-15:
            break
        small = abs(ln - lam) <= 1e-15
        u, g, lam = un, gn, ln
        if small:
            break
    return lam, u


def converge(Cu: np.ndarray, n: int, u0, alpha: float, tol: float = 1e-13, max_iter: int = 10000):
    """The local maximum SS-HOPM reaches from u0 (Sec. 3.1), converged: SS-HOPM
    until |delta lambda| <= tol or max_iter updates, then newton_finish.
    Returns (lambda, u, SS-HOPM updates)."""
    _, u, it, _ = sshopm(Cu, n, u0, alpha, tol, max_iter)
    lam, u = newton_finish(Cu, n, u)
    return lam, u, it


def newton_ascent(Cu: np.ndarray, n: int, u0: np.ndarray, steps: int, tol: float,
                  drop: float = 1e-6, halvings: int = 2):
    """Riemannian Newton iterations for max <C, u^{(x)n}> on the unit sphere.

    This is the search of the learned start (not in the paper; its parameters
    are part of that method's definition).  From u0, each step needs the tangent
    Hessian (n-1) E^T H E - lambda I to be negative definite.  A step that
    lowers lambda by more than ``drop`` (for C / ||C||_F, lambda <= 1) is
    halved, at most ``halvings`` times, and the search fails if it still does.
    The iteration has converged after a full step that changes lambda by at
    most ``tol``.  Returns (u, lambda, converged); when it fails or runs out of
    steps, converged is False.
    """
    u = np.asarray(u0, dtype=np.float64)
    u = u / np.linalg.norm(u)
    g = sym.contract_n_minus_1(Cu, u, n)
    lam = float(g @ u)
    for _ in range(steps):
        d = newton_direction(Cu, n, u, g, lam)
        if d is None:
            return u, lam, False
        t = 1.0
        for _h in range(halvings + 1):
            un = u + t * d
            un = un / np.linalg.norm(un)
            gn = sym.contract_n_minus_1(Cu, un, n)
            ln = float(gn @ un)
            if ln >= lam - drop:
                break
            t *= 0.5
        else:
            return u, lam, False
        done = t == 1.0 and abs(ln - lam) <= tol
        u, g, lam = un, gn, ln
        if done:
            return u, lam, True
    return u, lam, False


def newton_polish(Cu: np.ndarray, n: int, u: np.ndarray, steps: int = 2,
                  drop: float = 1e-7) -> np.ndarray:
    """Up to ``steps`` Newton steps on the sphere from u, each taken only where
    the tangent Hessian is negative definite and kept only if lambda does not
    fall by more than ``drop``.  The learned start's search ends its SS-HOPM
    continuation with these steps (part of that method's definition: the point
    they reach is the one its acceptance test looks at)."""
    u = np.asarray(u, dtype=np.float64)
    for _ in range(steps):
        g = sym.contract_n_minus_1(Cu, u, n)
        lam = float(g @ u)
        d = newton_direction(Cu, n, u, g, lam)
        if d is None:
            break
        un = u + d
        un = un / np.linalg.norm(un)
        if float(sym.contract_n_minus_1(Cu, un, n) @ un) < lam - drop:
            break
        u = un
    return u


def newton_step_length(Cu: np.ndarray, n: int, u: np.ndarray) -> float:
    """Length of the Riemannian Newton step at u (an estimate of the distance to
    the local maximum near u), or inf where the tangent Hessian is not negative
    definite (u is then not near a local maximum)."""
    u = np.asarray(u, dtype=np.float64)
    g = sym.contract_n_minus_1(Cu, u, n)
    d = newton_direction(Cu, n, u, g, float(g @ u))
    return np.inf if d is None else float(np.linalg.norm(d))


def certify(Cu: np.ndarray, n: int, u: np.ndarray, delta: float = 1e-2, steps: int = 4,
            drop: float = 1e-6, halvings: int = 2, grad_tol: float = 3e-5,
            curv_tol: float = 1e-3):
    """Certify u as near a local maximum (the learned start's acceptance test,
    part of that method's definition): the tangent gradient |g - lambda u| is
    at most grad_tol and the tangent Hessian's largest eigenvalue at most
    curv_tol (a critical point to rounding level that is not a minimum or a
    clear saddle), or the tangent Hessian is negative definite and the Newton
    step at u is at most delta long.  Otherwise a Newton step is taken
    (halved, at most ``halvings`` times, while lambda falls by more than
    ``drop``) and the test repeats, at most ``steps`` times; where the tangent
    Hessian is not negative definite, or a halved step still falls, u is not
    certified.  Returns (u, certified, the last step length measured; 0 when
    certified by the gradient)."""
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    length = np.inf
    for k in range(steps + 1):
        g = sym.contract_n_minus_1(Cu, u, n)
        lam = float(g @ u)
        E = tangent_basis(u)
        amax = float(np.linalg.eigvalsh(tangent_hessian(Cu, n, u, lam, E)).max())
        if np.linalg.norm(g - lam * u) <= grad_tol and amax <= curv_tol:
            return u, True, 0.0
        d = newton_direction(Cu, n, u, g, lam)
        if d is None:
            return u, False, np.inf
        length = float(np.linalg.norm(d))
        if length <= delta:
            return u, True, length
        if k == steps:
            break
        t = 1.0
        for _h in range(halvings + 1):
            un = u + t * d
            un = un / np.linalg.norm(un)
            if float(sym.contract_n_minus_1(Cu, un, n) @ un) >= lam - drop:
                break
            t *= 0.5
        else:
            return u, False, length
        u = un
    return u, False, length


def orient_multistart(Cv: np.ndarray, n: int, starts: np.ndarray, tol: float = 1e-13,
                      max_iter: int = 10000, shift: float | None = None):
    """Dominant eigenpair of one voxel's tensor from fixed starts (Sec. 3.1).

    Works on C / ||C||_F with the unfolding shift unless ``shift`` is given;
    from every start, the converged local maximum (``converge``: SS-HOPM to
    tol, then Newton to rounding level); the largest lambda wins, the first
    start on ties.  Returns (lambda, u, per-start lambdas, per-start
    directions, per-start SS-HOPM updates); lambdas are scaled back by
    ||C||_F.  A zero tensor gives lambda = 0, u = 0.
    """
    d = starts.shape[1]
    cn = float(sym.frobenius(Cv, n, d))
    if cn == 0.0:
        return (0.0, np.zeros(d), np.zeros(len(starts)), np.zeros((len(starts), d)),
                np.zeros(len(starts), int))
    Cu = np.asarray(Cv, dtype=np.float64) / cn
    alpha = unfolding_shift(Cu, n, d) if shift is None else shift
    _, U, its, _ = sshopm(Cu, n, starts, alpha, tol, max_iter)
    lams, us = [], []
    for u in U:
        lam, u = newton_finish(Cu, n, u)
        lams.append(lam)
        us.append(u)
    lams = np.array(lams)
    best = int(np.argmax(lams))            # first maximum on ties
    return cn * lams[best], canonical_sign(us[best]), cn * lams, np.array(us), np.array(its)


def sshopm_rate(Cv: np.ndarray, n: int, u: np.ndarray, alpha: float | None = None) -> float:
    """Linear convergence factor of SS-HOPM at a fixed point u of C / ||C||_F.

    The update's Jacobian on the tangent plane of u has eigenvalues
    ((n - 1) mu_j + alpha) / (lambda + alpha), mu_j the eigenvalues of
    C u^{n-2} restricted to that plane.  Values near 1 mean slow convergence
    and a maximiser that small perturbations of C move far.
    """
    d = len(u)
    cn = float(sym.frobenius(Cv, n, d))
    Cu = np.asarray(Cv, dtype=np.float64) / cn
    if alpha is None:
        alpha = unfolding_shift(Cu, n, d)
    u = np.asarray(u, dtype=np.float64) / np.linalg.norm(u)
    lam = float(sym.contract_n_minus_1(Cu, u, n) @ u)
    H = sym.contract_n_minus_2(Cu, u, n)
    E = tangent_basis(u)
    mu = np.linalg.eigvalsh(E.T @ H @ E)
    return float(np.max(np.abs((n - 1) * mu + alpha)) / (lam + alpha))


def axis_distance_deg(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """The angle metric of the form: arccos|u.v| for axes (d' = 3), the
    rotation distance 2 arccos|q1.q2| for quaternions (d' = 4, Sec. 4.1)."""
    u = np.asarray(u, dtype=np.float64)
    return quat_angle_deg(u, v) if u.shape[-1] == 4 else angle_deg(u, v)


def orientation_margin(lams: np.ndarray, us: np.ndarray, best_u: np.ndarray,
                       sep_deg: float = 5.0) -> float:
    """lambda_best minus the best lambda of starts that ended more than sep_deg away.

    A small margin means two distinct local maxima are nearly tied and either
    answer is correct; such voxels are reported as ambiguous.
    """
    far = axis_distance_deg(us, best_u[None, :]) > sep_deg
    if not np.any(far):
        return np.inf
    return float(np.max(lams) - np.max(lams[far]))


def fibonacci_sphere(n: int) -> np.ndarray:
    """n near-uniform points on S^2 (golden-angle spiral)."""
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    phi = np.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def spiral_s3(n: int) -> np.ndarray:
    """n near-uniform points on S^3: the super-Fibonacci spiral (Alexa 2022),
    s = i + 1/2, (sqrt(s/n) sin a, sqrt(s/n) cos a, sqrt(1-s/n) sin b,
    sqrt(1-s/n) cos b) with a = 2 pi s / sqrt(2), b = 2 pi s / psi, psi^4 = psi + 4."""
    psi = 1.533751168755204288118041
    s = np.arange(n) + 0.5
    r, R = np.sqrt(s / n), np.sqrt(1.0 - s / n)
    a, b = 2.0 * np.pi * s / math.sqrt(2.0), 2.0 * np.pi * s / psi
    return np.stack([r * np.sin(a), r * np.cos(a), R * np.sin(b), R * np.cos(b)], axis=1)


def reference_maxima(Cv: np.ndarray, n: int, grid: int = 20000, polish: int = 8,
                     sep_deg: float = 5.0, dprime: int = 3):
    """Global maximiser by dense sampling, then convergence from the best points.

    Evaluates <C, u^{(x)n}> on a near-uniform point set (Fibonacci sphere for
    d' = 3, super-Fibonacci spiral on S^3 for d' = 4), converges (``converge``)
    from the best grid points that lie more than sep_deg apart, and returns
    (lambda*, u*, lambda_2): lambda_2 is the best converged maximum more than
    sep_deg from u* (up to sign), or -inf.
    """
    pts = fibonacci_sphere(grid) if dprime == 3 else spiral_s3(grid)
    vals = sym.weights(n, dprime) * sym.monomials(pts, n) @ np.asarray(Cv, dtype=np.float64)
    order = np.argsort(-vals)
    chosen = []
    for i in order:
        if all(axis_distance_deg(pts[i], pts[j]) > sep_deg for j in chosen):
            chosen.append(i)
        if len(chosen) >= polish:
            break
    cn = float(sym.frobenius(Cv, n, dprime))
    if cn == 0.0:
        return 0.0, np.zeros(dprime), -np.inf
    Cu = np.asarray(Cv, dtype=np.float64) / cn
    alpha = unfolding_shift(Cu, n, dprime)
    found = []
    for i in chosen:
        lam, u, _ = converge(Cu, n, pts[i], alpha)
        found.append((lam * cn, canonical_sign(u)))
    found.sort(key=lambda t: -t[0])
    lam1, u1 = found[0]
    lam2 = -np.inf
    for lam, u in found[1:]:
        if axis_distance_deg(u, u1) > sep_deg:
            lam2 = lam
            break
    return lam1, u1, lam2


def angle_deg(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Axis angle arccos|u.v| in degrees (u and -u are the same axis)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    c = np.abs(np.sum(u * v, axis=-1)) / (np.linalg.norm(u, axis=-1) * np.linalg.norm(v, axis=-1))
    return np.degrees(np.arccos(np.clip(c, 0.0, 1.0)))


def quat_angle_deg(q1: np.ndarray, q2: np.ndarray) -> np.ndarray:
    """Rotation distance 2 arccos|q1.q2| in degrees (Sec. 4.1), unit quaternions."""
    q1 = np.asarray(q1, dtype=np.float64)
    q2 = np.asarray(q2, dtype=np.float64)
    c = np.abs(np.sum(q1 * q2, axis=-1)) / (np.linalg.norm(q1, axis=-1) * np.linalg.norm(q2, axis=-1))
    return np.degrees(2.0 * np.arccos(np.clip(c, 0.0, 1.0)))


# ----------------------------------------------------------------------------
# peaks
# ----------------------------------------------------------------------------


def find_peaks(score_map: np.ndarray, valid_lo, valid_hi, top_p: int, min_dist: float):
    """Greedy Find Peaks (Sec. 3.4): P highest scores, pairwise >= min_dist apart.

    Candidates are the valid voxels [valid_lo, valid_hi] (inclusive, z, y, x);
    order is descending score, then ascending linear index z*Y*X + y*X + x.
    A candidate is kept if its distance to every kept peak is >= min_dist.
    Returns (positions (P', 3) int64 z, y, x; scores (P',)).
    """
    Z, Y, X = score_map.shape
    z0, y0, x0 = valid_lo
    z1, y1, x1 = valid_hi
    sub = score_map[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1]
    zz, yy, xx = np.meshgrid(np.arange(z0, z1 + 1), np.arange(y0, y1 + 1),
                             np.arange(x0, x1 + 1), indexing="ij")
    lin = (zz * Y * X + yy * X + xx).ravel()
    vals = sub.ravel()
    order = np.lexsort((lin, -vals))
    kept = np.zeros((0, 3))
    out_pos, out_val = [], []
    d2 = float(min_dist) ** 2
    for i in order:
        if len(out_pos) >= top_p:
            break
        p = np.array([lin[i] // (Y * X), (lin[i] // X) % Y, lin[i] % X], dtype=np.float64)
        if len(kept) and np.min(np.sum((kept - p) ** 2, axis=1)) < d2:
            continue
        kept = np.vstack([kept, p])
        out_pos.append(p.astype(np.int64))
        out_val.append(vals[i])
    return np.array(out_pos, dtype=np.int64).reshape(-1, 3), np.array(out_val)


# ----------------------------------------------------------------------------
# position refinement (TTM-ref, Alg. 3)
# ----------------------------------------------------------------------------


def sphere_offsets(rs: float) -> np.ndarray:
    """Integer offsets (dz, dy, dx) with |d| <= rs, the zero offset first, the
    others in lexicographic (dz, dy, dx) order.  The order fixes which voxel
    wins a tie in the refinement."""
    R = int(math.floor(rs))
    out = [(0, 0, 0)]
    for dz in range(-R, R + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                if (dz, dy, dx) != (0, 0, 0) and dz * dz + dy * dy + dx * dx <= rs * rs:
                    out.append((dz, dy, dx))
    return np.array(out, dtype=np.int64)


def lncc_at(g: np.ndarray, w: np.ndarray, tn: np.ndarray, x, q) -> float:
    """c(x, R(q)) = w(x) (g * t'_R)(x) at one voxel (Eq. lncc): t' rotated by
    R(q) (trilinear pull-back, zero outside the box) dotted with the template
    window of g at x."""
    L = tn.shape[0]
    c = L // 2
    z, y, x0 = (int(v) for v in x)
    tq = rotate_template(tn, quat_to_matrix(np.asarray(q, dtype=np.float64)))
    patch = np.asarray(g[z - c:z - c + L, y - c:y - c + L, x0 - c:x0 - c + L], dtype=np.float64)
    return float(w[z, y, x0]) * float(np.sum(patch * tq))


def refine_positions(g: np.ndarray, w: np.ndarray, tn: np.ndarray, field_of, orient_of,
                     peaks: np.ndarray, rs: float = 3.0):
    """TTM-ref (Sec. 3.3, Alg. 3): for each peak x^i, the rotation R_opt from
    C(x^i) and its LNCC c = c(x^i, R_opt) start the search (x~ = x^i); then for
    every other voxel x^j of the sphere |x^j - x^i| <= r_s (sphere_offsets
    order) the rotation R from C(x^j) and c~ = c(x^j, R); x^j replaces the
    current best when c~ > c.  Readings: the sphere of the loop is V_{x^i}
    (the printed index is garbled); x~ starts at x^i; voxels whose template
    window leaves the volume (outside the valid region) are skipped.

    field_of(x) -> C(x) (K,) and orient_of(C) -> unit quaternion (4,) supply
    the tensor field and the optimal rotation (d' = 4).  Returns per peak:
    (refined position (3,), its quaternion, its LNCC, the peak's own
    quaternion, the peak's LNCC)."""
    L = tn.shape[0]
    c = L // 2
    lo = np.array([c, c, c])
    hi = np.array([d - L + c for d in g.shape])
    offs = sphere_offsets(rs)
    out = []
    for p in np.asarray(peaks, dtype=np.int64):
        q0 = orient_of(field_of(p))
        c0 = lncc_at(g, w, tn, p, q0)
        best = (p.copy(), q0, c0)
        for d in offs[1:]:
            xj = p + d
            if np.any(xj < lo) or np.any(xj > hi):
                continue
            qj = orient_of(field_of(xj))
            cj = lncc_at(g, w, tn, xj, qj)
            if cj > best[2]:
                best = (xj, qj, cj)
        out.append((best[0], best[1], best[2], q0, c0))
    return out


# ----------------------------------------------------------------------------
# rotation-sampled template matching (the comparison method; tests only)
# ----------------------------------------------------------------------------


def brute_force_tm(g: np.ndarray, w: np.ndarray, tn: np.ndarray, quats: np.ndarray) -> np.ndarray:
    """c(x, R_q) = w(x) (g * t'_q)(x) on the valid region (Eq. lncc), shape (N_q, Vz, Vy, Vx)."""
    L = tn.shape[0]
    c = L // 2
    rot = np.stack([rotate_template(tn, quat_to_matrix(q)) for q in quats])
    raw = correlate_valid(g, rot)
    Vz, Vy, Vx = raw.shape[1:]
    return raw * w[None, c:c + Vz, c:c + Vy, c:c + Vx]
