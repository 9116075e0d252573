"""Pins of the TTM oracle: closed forms, invariants, textbook routines, brute force."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.signal as ss

import synth
from oracle import rotations as rot
from oracle import sym, ttm


def _tiny(seed=7, D=32, L=12, r=5.0, copies=2, amp=3.0):
    return synth.make_tomogram("tiny", (D, D, D), L=L, n_blobs=3, n_copies=copies, min_sep=L,
                               mask_radius=r, degree=4, seed=seed, snr=None, wedge=False,
                               copy_amplitude=amp)


# ---------------------------------------------------------------- P-1 filter
def test_filter_impulse_and_frequency_response():
    a = 0.2
    imp = np.zeros((7, 7, 7))
    imp[3, 3, 3] = 1.0
    g = ttm.prefilter_template(imp, a)
    taps = np.array([a, 1 - 2 * a, a])
    want = np.zeros((7, 7, 7))
    want[2:5, 2:5, 2:5] = taps[:, None, None] * taps[None, :, None] * taps[None, None, :]
    assert np.allclose(g, want)
    # 1D response 1 + a(z + 1/z - 2) on the unit circle = 1 - 4a sin^2(w/2) in [1 - 4a, 1]
    w = np.linspace(0, np.pi, 101)
    H = np.array([np.sum(taps * np.exp(-1j * k * np.array([-1, 0, 1]))) for k in w])
    assert np.allclose(H.imag, 0, atol=1e-15)
    assert np.allclose(H.real, 1 - 4 * a * np.sin(w / 2) ** 2)
    assert H.real.min() == pytest.approx(0.2) and H.real.max() == pytest.approx(1.0)


def test_prefilter_volume_matches_scipy_and_constants():
    rng = np.random.default_rng(0)
    f = rng.standard_normal((9, 10, 11))
    taps = np.array([0.2, 0.6, 0.2])
    want = f
    for ax in range(3):
        want = ndi.correlate1d(want, taps, axis=ax, mode="nearest")
    assert np.allclose(ttm.prefilter_volume(f), want, atol=1e-13)
    assert np.allclose(ttm.prefilter_volume(np.full((5, 6, 7), 3.25)), 3.25, atol=1e-14)


def test_prefilter_box_equals_volume_filter():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((20, 21, 22))
    g = ttm.prefilter_volume(f)
    for lo, hi in [((0, 0, 0), (5, 6, 7)), ((3, 4, 5), (20, 21, 22)), ((7, 2, 9), (15, 12, 19))]:
        assert np.allclose(ttm.prefilter_box(f, lo, hi), g[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]])


# ---------------------------------------------------------------- P-2 template
def test_template_zero_normalised():
    rng = np.random.default_rng(2)
    for L, r in [(12, 5.0), (16, 7.0), (15, 6.5)]:
        t = rng.standard_normal((L, L, L)) + 2.0
        tn = ttm.normalize_template(t, r)
        m = ttm.ball_mask(L, r)
        assert abs(tn.sum()) < 1e-12
        assert np.sum(tn * tn) == pytest.approx(1.0, abs=1e-12)
        assert np.all(tn[m == 0] == 0)


def test_lncc_bounded_by_one():
    w = _tiny()
    g = ttm.prefilter_volume(w.volume)
    m = ttm.ball_mask(12, 5.0)
    wm = ttm.local_normalization(g, m)
    tn = ttm.normalize_template(w.template, 5.0)
    c = ttm.brute_force_tm(g, wm, tn, synth.rotation_samples(1))
    assert np.abs(c).max() <= 1.0 + 1e-12
    # exact copy at the planted pose is found at the planted centre
    R = w.rotations[0]
    q = _mat2quat(R)
    c0 = ttm.brute_force_tm(g, wm, tn, q[None])[0]
    lo, _ = ttm.valid_range(32, 12)
    z, y, x = w.centres[0]
    assert np.unravel_index(np.argmax(c0), c0.shape) == (z - lo, y - lo, x - lo)


def _mat2quat(R):
    w = math.sqrt(max(0.0, 1 + R[0, 0] + R[1, 1] + R[2, 2])) / 2
    x = math.copysign(math.sqrt(max(0.0, 1 + R[0, 0] - R[1, 1] - R[2, 2])) / 2, R[2, 1] - R[1, 2])
    y = math.copysign(math.sqrt(max(0.0, 1 - R[0, 0] + R[1, 1] - R[2, 2])) / 2, R[0, 2] - R[2, 0])
    z = math.copysign(math.sqrt(max(0.0, 1 - R[0, 0] - R[1, 1] + R[2, 2])) / 2, R[1, 0] - R[0, 1])
    return np.array([w, x, y, z])


# ---------------------------------------------------------------- P-12 correlation
def test_correlate_valid_matches_scipy_direct():
    rng = np.random.default_rng(3)
    g = rng.standard_normal((14, 13, 15))
    k = rng.standard_normal((2, 5, 5, 5))
    out = ttm.correlate_valid(g, k)
    for i in range(2):
        want = ss.correlate(g, k[i], mode="valid", method="direct")
        assert np.allclose(out[i], want, atol=1e-12)


def test_correlation_theorem_small():
    # FFT correlation (numpy, FP64) equals the direct sums on the valid region
    rng = np.random.default_rng(4)
    D, L = 16, 6
    g = rng.standard_normal((D, D, D))
    k = rng.standard_normal((L, L, L))
    kp = np.zeros((D, D, D))
    kp[:L, :L, :L] = k
    fft = np.real(np.fft.ifftn(np.fft.fftn(g) * np.conj(np.fft.fftn(kp))))
    direct = ttm.correlate_valid(g, k[None])[0]
    V = D - L + 1
    assert np.allclose(fft[:V, :V, :V], direct, atol=1e-11)


# ---------------------------------------------------------------- P-11 local variance
def test_local_variance_textbook_and_invariances():
    rng = np.random.default_rng(5)
    D, L, r = 18, 8, 3.0
    f = rng.standard_normal((D, D, D))
    g = ttm.prefilter_volume(f)
    m = ttm.ball_mask(L, r)
    M = m.sum()
    var = ttm.local_variance(g, m)
    # textbook: M times the population variance of the window voxels inside the ball
    win = np.lib.stride_tricks.sliding_window_view(g, (L, L, L))
    sel = m.astype(bool)
    for (z, y, x) in [(0, 0, 0), (3, 7, 2), (10, 10, 10)]:
        vals = win[z, y, x][sel]
        assert var[z, y, x] == pytest.approx(M * np.var(vals), rel=1e-10)
    w1 = ttm.local_normalization(g, m)
    w2 = ttm.local_normalization(ttm.prefilter_volume(f + 17.0), m)
    assert np.allclose(w1, w2, rtol=1e-8)
    c0, c1 = ttm.valid_range(D, L)
    assert np.all(w1[:c0] == 0) and np.all(w1[c1 + 1:] == 0)
    assert np.all(w1[c0:c1 + 1, c0:c1 + 1, c0:c1 + 1] > 0)
    wc = ttm.local_normalization(ttm.prefilter_volume(np.full((D, D, D), 2.5)), m)
    assert np.all(wc == 0)


def test_field_and_score_invariant_under_intensity_scale():
    """Eq. norm_f with Eq. tcc: for f -> a f (a > 0) the prefiltered image and the
    correlations scale by a and w by 1/a (the guard scales with the variance), so C
    and its score are unchanged."""
    w = _tiny(seed=12, D=24, L=10, r=4.0, copies=1)
    m = ttm.ball_mask(10, 4.0)
    tn = ttm.normalize_template(w.template, 4.0)
    T = ttm.tensor_template(tn, synth.rotation_samples(2), 4)

    def field(f):
        g = ttm.prefilter_volume(f)
        return ttm.tensor_field(g, ttm.local_normalization(g, m), T)

    f = w.volume.astype(np.float64)   # scaled in FP64, so the only rounding is the oracle's
    C1 = field(f)
    for a in (1e-3, 7.5):
        Ca = field(a * f)
        assert np.allclose(Ca, C1, rtol=1e-9, atol=1e-12 * np.abs(C1).max())
        assert np.allclose(ttm.score(Ca, 4), ttm.score(C1, 4), rtol=1e-9)


# ---------------------------------------------------------------- P-3 TTM vs TM identity
@pytest.mark.parametrize("n,dprime", [(4, 3), (2, 3), (2, 4)])
def test_field_equals_rotation_average_of_tm(n, dprime):
    w = _tiny(seed=11, D=24, L=10, r=4.0, copies=1)
    g = ttm.prefilter_volume(w.volume)
    m = ttm.ball_mask(10, 4.0)
    wm = ttm.local_normalization(g, m)
    tn = ttm.normalize_template(w.template, 4.0)
    Q = synth.rotation_samples(3)                    # 72 rotations
    T = ttm.tensor_template(tn, Q, n, dprime)
    C = ttm.tensor_field(g, wm, T)
    c = ttm.brute_force_tm(g, wm, tn, Q)            # (Nq, V, V, V)
    rng = np.random.default_rng(6)
    V = np.stack([ttm.direction_of(q, dprime) for q in Q])
    for _ in range(3):
        u = rng.standard_normal(dprime)
        lhs = np.tensordot(sym.weights(n, dprime) * sym.monomials(u, n), C, axes=(0, 0))
        rhs = np.tensordot((V @ u) ** n, c, axes=(0, 0)) / len(Q)
        assert np.allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max() + 1e-14)


def test_trace_reduces_to_averaged_template_correlation():
    # P-7: sum over pairwise traces <C, E> with E.v^n = |v|^n equals w (g * t_bar),
    # t_bar the rotation-averaged template; n = 0 gives the same field directly.
    w = _tiny(seed=12, D=22, L=10, r=4.0, copies=1)
    g = ttm.prefilter_volume(w.volume)
    m = ttm.ball_mask(10, 4.0)
    wm = ttm.local_normalization(g, m)
    tn = ttm.normalize_template(w.template, 4.0)
    Q = synth.rotation_samples(2)
    tbar = np.mean([rot.rotate_template(tn, rot.quat_to_matrix(q)) for q in Q], axis=0)
    c = 5
    want = ss.correlate(g, tbar, mode="valid", method="direct")
    V = want.shape[0]
    want = want * wm[c:c + V, c:c + V, c:c + V]
    C0 = ttm.tensor_field(g, wm, ttm.tensor_template(tn, Q, 0))
    assert np.allclose(C0[0], want, atol=1e-12)
    n = 4
    C4 = ttm.tensor_field(g, wm, ttm.tensor_template(tn, Q, n))
    # trace: sum_{i,j} C_{iijj} (full tensor); built from the full expansion per voxel
    tr = np.zeros(C4.shape[1:])
    idx = sym.index_of(n, 3)
    for i in range(3):
        for j in range(3):
            cnt = [0, 0, 0]
            cnt[i] += 2
            cnt[j] += 2
            tr += C4[idx[tuple(cnt)]]
    assert np.allclose(tr, want, atol=1e-12)


# ---------------------------------------------------------------- P-5 equivariance
def test_tensor_template_octahedral_equivariance():
    L, r, n = 13, 4.0, 4
    rng = np.random.default_rng(8)
    t = ndi.gaussian_filter(rng.standard_normal((L, L, L)), 1.0)
    tn = ttm.normalize_template(t, r)
    Q = synth.rotation_samples(2)
    T = ttm.tensor_template(tn, Q, n)
    c = L // 2
    idx = np.arange(L) - c
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    P = np.stack([xx, yy, zz], axis=-1)
    for G in rot.cube_group()[:8]:
        # T(c + G (p - c)) = G^{(x)n} . T(p)
        dst = np.rint(P @ G.T).astype(int) + c
        lhs = T[:, dst[..., 2], dst[..., 1], dst[..., 0]]
        rhs = np.stack([sym.rotate(T[:, z, y, x], G, n) for z in range(L) for y in range(L)
                        for x in range(L)], axis=1).reshape(T.shape)
        assert np.allclose(lhs, rhs, atol=1e-12)


def test_tensor_field_octahedral_equivariance():
    D, L, r, n = 21, 9, 3.5, 4
    rng = np.random.default_rng(9)
    f = rng.standard_normal((D, D, D))
    t = ndi.gaussian_filter(rng.standard_normal((L, L, L)), 1.0)
    tn = ttm.normalize_template(t, r)
    T = ttm.tensor_template(tn, synth.rotation_samples(2), n)
    m = ttm.ball_mask(L, r)

    def field(vol):
        g = ttm.prefilter_volume(vol)
        return ttm.tensor_field(g, ttm.local_normalization(g, m), T)

    C = field(f)
    cv = (D - 1) / 2
    idx = np.arange(D) - cv
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    P = np.stack([xx, yy, zz], axis=-1)
    c0 = L // 2
    V = D - L + 1
    for G in rot.cube_group()[1:6]:
        # f'(x) = f(cv + G^T (x - cv)): an exact voxel permutation
        src = np.rint(P @ G + cv).astype(int)
        fr = f[src[..., 2], src[..., 1], src[..., 0]]
        Cr = field(fr)
        # C'(cv + G (x - cv)) = G^{(x)n} C(x) for valid x
        for (z, y, x) in [(0, 0, 0), (3, 5, 7), (V - 1, 2, V - 1), (6, 6, 6)]:
            p = np.array([x + c0, y + c0, z + c0]) - cv
            q = np.rint(G @ p + cv).astype(int) - c0
            got = Cr[:, q[2], q[1], q[0]]
            want = sym.rotate(C[:, z, y, x], G, n)
            assert np.allclose(got, want, atol=1e-12)


# ---------------------------------------------------------------- P-8 .. P-10 orientation
@pytest.mark.parametrize("n", [4, 6])
def test_rank_one_recovers_direction(n):
    rng = np.random.default_rng(10)
    starts = synth.start_vectors().astype(np.float64)
    for _ in range(5):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        lam0 = rng.uniform(0.5, 3.0)
        C = lam0 * sym.monomials(v, n)
        lam, u, *_ = ttm.orient_multistart(C, n, starts, tol=1e-14, max_iter=5000)
        assert lam == pytest.approx(lam0, rel=1e-9)
        assert ttm.angle_deg(u, v) < 1e-4
        assert ttm.score(C, n) == pytest.approx(lam0)


def test_degree_two_is_symmetric_eigenproblem():
    rng = np.random.default_rng(11)
    starts = synth.start_vectors().astype(np.float64)
    for _ in range(10):
        A = rng.standard_normal((3, 3))
        A = A + A.T
        C = np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]])
        assert np.allclose(sym.to_full(C, 2, 3), A)
        ev, evec = np.linalg.eigh(A)
        lam, u, *_ = ttm.orient_multistart(C, 2, starts, tol=1e-15, max_iter=20000)
        assert lam == pytest.approx(ev[-1], rel=1e-9)
        assert ttm.angle_deg(u, evec[:, -1]) < 1e-4


@pytest.mark.parametrize("n", [4, 6])
def test_sshopm_monotone_fixed_point_and_bracket(n):
    rng = np.random.default_rng(12)
    for _ in range(6):
        C = rng.standard_normal(sym.n_components(n, 3))
        cn = ttm.score(C, n)
        Cu = C / cn
        alpha = ttm.unfolding_shift(Cu, n, 3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        lam_prev = -np.inf
        for _ in range(3000):
            g = sym.contract_n_minus_1(Cu, u, n)
            lam = g @ u
            assert lam >= lam_prev - 1e-13
            lam_prev = lam
            v = g + alpha * u
            u = v / np.linalg.norm(v)
        g = sym.contract_n_minus_1(Cu, u, n)
        assert np.linalg.norm(g - (g @ u) * u) < 1e-8
        lam, *_ = ttm.orient_multistart(C, n, synth.start_vectors(count=64).astype(np.float64),
                                        tol=1e-13, max_iter=20000)
        # spectral-norm bracket: ||C||_F / 2^{n-1} <= max|lambda| <= ||C||_F (Sec. 3.2)
        lam_min, *_ = ttm.orient_multistart(-C, n, synth.start_vectors(count=64).astype(np.float64),
                                            tol=1e-13, max_iter=20000)
        spec = max(abs(lam), abs(lam_min))
        assert cn / 2 ** (n - 1) <= spec + 1e-12
        assert spec <= cn + 1e-12


def test_orientation_rotates_with_tensor():
    # P-4: lambda(G.C) = lambda(C) and u(G.C) = G u(C)
    rng = np.random.default_rng(13)
    n = 6
    starts = synth.start_vectors(count=32).astype(np.float64)
    for _ in range(4):
        v = rng.standard_normal(3)
        C = sym.monomials(v / np.linalg.norm(v), n) * 2 + 0.3 * rng.standard_normal(28)
        G, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        if np.linalg.det(G) < 0:
            G[:, 0] *= -1
        lam, u, *_ = ttm.orient_multistart(C, n, starts, tol=1e-14, max_iter=20000)
        lam2, u2, *_ = ttm.orient_multistart(sym.rotate(C, G, n), n, starts, tol=1e-14, max_iter=20000)
        assert lam2 == pytest.approx(lam, rel=1e-9)
        assert ttm.angle_deg(u2, G @ u) < 1e-4


def test_reference_maxima_agree_with_multistart():
    rng = np.random.default_rng(14)
    n = 6
    for _ in range(3):
        C = rng.standard_normal(28)
        lam, u, *_ = ttm.orient_multistart(C, n, synth.start_vectors(count=64).astype(np.float64),
                                           tol=1e-14, max_iter=20000)
        lr, ur, l2 = ttm.reference_maxima(C, n, grid=4000)
        assert lr >= lam - 1e-9
        if lr - lam < 1e-9:
            assert ttm.angle_deg(u, ur) < 1e-3


# ---------------------------------------------------------------- P-13 peaks
def _greedy_brute(vals, lin, shape, P, D):
    order = sorted(range(len(vals)), key=lambda i: (-vals[i], lin[i]))
    Y, X = shape[1], shape[2]
    out = []
    for i in order:
        if len(out) >= P:
            break
        p = np.array([lin[i] // (Y * X), (lin[i] // X) % Y, lin[i] % X])
        if all(np.sum((p - q) ** 2) >= D * D for q in out):
            out.append(p)
    return np.array(out)


def test_find_peaks_brute_force_with_ties():
    rng = np.random.default_rng(15)
    s = np.round(rng.uniform(0, 1, (12, 13, 14)), 2)       # many exact ties
    lo, hi = (2, 1, 3), (10, 11, 12)
    pk, pv = ttm.find_peaks(s, lo, hi, 15, 3.0)
    zz, yy, xx = np.meshgrid(range(lo[0], hi[0] + 1), range(lo[1], hi[1] + 1),
                             range(lo[2], hi[2] + 1), indexing="ij")
    lin = (zz * 13 * 14 + yy * 14 + xx).ravel()
    vals = s[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1].ravel()
    want = _greedy_brute(vals, lin, s.shape, 15, 3.0)
    assert np.array_equal(pk, want)
    assert np.array_equal(pv, s[pk[:, 0], pk[:, 1], pk[:, 2]])


def test_find_peaks_filtered_rounds_give_the_same_peaks():
    """Sec. 3.4's rule decides a voxel only from the peaks kept before it, so a
    voxel within D of a peak kept from a prefix of the visiting order is never
    kept; dropping such voxels from the rest of the order (several rounds of a
    short walk and a filter, with P out of reach so every voxel is visited)
    must leave the peaks unchanged."""
    rng = np.random.default_rng(23)
    s = np.round(rng.uniform(0, 1, (14, 16, 18)), 2)      # many exact ties
    lo, hi = (1, 1, 2), (12, 15, 16)
    P, D = 500, 3.5
    pk, pv = ttm.find_peaks(s, lo, hi, P, D)
    assert len(pk) < P                                     # every voxel is walked
    zz, yy, xx = np.meshgrid(range(lo[0], hi[0] + 1), range(lo[1], hi[1] + 1),
                             range(lo[2], hi[2] + 1), indexing="ij")
    lin = (zz * 16 * 18 + yy * 18 + xx).ravel()
    vals = s[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1].ravel()
    order = np.lexsort((lin, -vals))
    pos = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], 1)[order]
    kept, lst, walk = [], pos, 64
    for last in (False, False, False, True):
        n = len(lst) if last else min(walk, len(lst))
        for p in lst[:n]:
            if all(np.sum((p - q) ** 2) >= D * D for q in kept):
                kept.append(p)
        rest = lst[n:]
        if len(rest) and kept:
            d2 = np.min(np.sum((rest[:, None, :] - np.array(kept)[None]) ** 2, axis=-1), axis=1)
            rest = rest[d2 >= D * D]
        lst = rest
    assert np.array_equal(np.array(kept), pk)


def test_planted_copies_recovered_at_high_snr():
    w = synth.make_tomogram("p", (48, 48, 48), L=16, n_blobs=3, n_copies=4, min_sep=20,
                            mask_radius=7.0, degree=4, seed=21, snr=None, wedge=False,
                            copy_amplitude=20.0)
    g = ttm.prefilter_volume(w.volume)
    m = ttm.ball_mask(16, 7.0)
    wm = ttm.local_normalization(g, m)
    tn = ttm.normalize_template(w.template, 7.0)
    T = ttm.tensor_template(tn, synth.rotation_samples(10), 4)
    C = ttm.tensor_field(g, wm, T)
    s = ttm.score(C, 4)
    lo, hi = ttm.valid_range(48, 16)
    smap = np.zeros(g.shape)
    smap[lo:hi + 1, lo:hi + 1, lo:hi + 1] = s
    pk, _ = ttm.find_peaks(smap, (lo,) * 3, (hi,) * 3, len(w.centres), 14.0)
    # every planted copy has a peak within the mask radius (the Frobenius score is
    # a position proxy that may shift by a few voxels, Sec. 4.1, Table 1)
    for c in w.centres:
        d = np.min(np.linalg.norm(pk - c, axis=1))
        assert d <= 7.0


def test_sshopm_rate_predicts_convergence():
    # the measured error ratio of late iterates approaches the predicted factor
    rng = np.random.default_rng(31)
    n = 6
    C = rng.standard_normal(28)
    Cu = C / ttm.score(C, n)
    alpha = ttm.unfolding_shift(Cu, n, 3)
    lam, u_star, _, _ = ttm.sshopm(Cu, n, synth.start_vectors()[0], alpha, -1.0, 5000)
    rate = ttm.sshopm_rate(C, n, u_star, alpha)
    assert 0 <= rate < 1
    u = synth.start_vectors()[0].astype(np.float64)
    errs = []
    for _ in range(400):
        v = sym.contract_n_minus_1(Cu, u, n) + alpha * u
        u = v / np.linalg.norm(v)
        errs.append(np.linalg.norm(u - u_star))
    e = np.array(errs)
    k = np.where(e > 1e-7)[0][-5]
    assert e[k + 1] / e[k] == pytest.approx(rate, abs=0.02)


def test_newton_finish_converges_quadratically_to_the_sshopm_maximum():
    rng = np.random.default_rng(41)
    n = 6
    for _ in range(5):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        C = sym.monomials(v, n) + 0.2 * rng.standard_normal(28)
        Cu = C / ttm.score(C, n)
        alpha = ttm.unfolding_shift(Cu, n, 3)
        _, u_star, _, _ = ttm.sshopm(Cu, n, v, alpha, -1.0, 20000)
        u0 = u_star + 0.02 * np.cross(u_star, rng.standard_normal(3))
        u0 /= np.linalg.norm(u0)
        e0 = np.linalg.norm(u0 - u_star)
        _, u1 = ttm.newton_finish(Cu, n, u0, max_steps=1)
        _, u2 = ttm.newton_finish(Cu, n, u0, max_steps=2)
        e1, e2 = np.linalg.norm(u1 - u_star), np.linalg.norm(u2 - u_star)
        assert e1 < 50 * e0 ** 2 and e2 < max(50 * e1 ** 2, 1e-12)
        tb = ttm.tangent_basis(u_star)
        assert np.allclose(tb.T @ tb, np.eye(2)) and np.allclose(tb.T @ u_star, 0)


@pytest.mark.parametrize("d", [3, 4])
def test_converge_reaches_the_sshopm_fixed_point(d):
    """P-9: the converged answer is a fixed point of SS-HOPM to rounding level,
    the same one a very long SS-HOPM run reaches, and lambda never falls."""
    rng = np.random.default_rng(42)
    st = synth.start_vectors(dim=d).astype(np.float64)
    for n in (4, 6) if d == 3 else (2, 4):
        for _ in range(3):
            C = rng.standard_normal(sym.n_components(n, d))
            lam, u, lams, us, its = ttm.orient_multistart(C, n, st)
            cn = ttm.score(C, n, d)
            Cu = C / cn
            for lk, uk in zip(lams, us):
                g = sym.contract_n_minus_1(Cu, uk, n)
                assert np.linalg.norm(g - (g @ uk) * uk) < 1e-10
                assert lk == pytest.approx(cn * (g @ uk), rel=1e-12)
            alpha = ttm.unfolding_shift(Cu, n, d)
            best = int(np.argmax(lams))
            lam2, u2, _, _ = ttm.sshopm(Cu, n, st[best], alpha, 1e-16, 200000)
            assert lam == pytest.approx(cn * lam2, rel=1e-9)
            assert ttm.axis_distance_deg(u, u2) < 1e-3


def test_newton_ascent_reaches_eigenvectors_and_refuses_non_maxima():
    rng = np.random.default_rng(43)
    # n = 2: <C, u^2> = u^T A u, whose maximisers on the sphere are the top
    # eigenvectors of A (numpy.linalg.eigh)
    for _ in range(5):
        A = rng.standard_normal((3, 3))
        A = A + A.T
        C = np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]])   # graded-lex, n = 2
        w, V = np.linalg.eigh(A)
        top, bottom = V[:, 2], V[:, 0]
        u0 = top + 0.05 * rng.standard_normal(3)
        u, lam, ok = ttm.newton_ascent(C, 2, u0, 8, 1e-12)
        assert ok and lam == pytest.approx(w[2], rel=1e-10) and ttm.angle_deg(u, top) < 1e-6
        # from near the bottom eigenvector the tangent Hessian is positive definite: refused
        u, lam, ok = ttm.newton_ascent(C, 2, bottom + 0.01 * rng.standard_normal(3), 8, 1e-12)
        assert not ok
    # rank one: C = v^n has its maximum lambda = 1 at u = +-v
    for n in (4, 6):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        C = sym.monomials(v, n)
        u0 = v + 0.08 * np.cross(v, rng.standard_normal(3))
        u, lam, ok = ttm.newton_ascent(C, n, u0, 8, 1e-14)
        assert ok and lam == pytest.approx(1.0, abs=1e-12) and ttm.angle_deg(u, v) < 1e-6


def test_newton_ascent_from_near_starts_matches_sshopm_with_polish():
    rng = np.random.default_rng(44)
    n = 6
    agree = total = 0
    for _ in range(60):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        C = sym.monomials(v, n) + 0.3 * rng.standard_normal(28)
        Cu = C / ttm.score(C, n)
        alpha = ttm.unfolding_shift(Cu, n, 3)
        _, u_s, _, _ = ttm.sshopm(Cu, n, v, alpha, 1e-13, 20000)
        w = rng.standard_normal(3)
        w -= (w @ u_s) * u_s
        u0 = np.cos(np.radians(2.0)) * u_s + np.sin(np.radians(2.0)) * w / np.linalg.norm(w)
        u, lam, ok = ttm.newton_ascent(Cu, n, u0, 5, 1e-5)
        if ok:
            total += 1
            # the Newton answer is a critical point up to the stopping rule: the
            # last step changed lambda by <= 1e-5, i.e. the previous error was
            # ~ sqrt(1e-5) and the quadratic step leaves ~ 1e-5 of it
            g = sym.contract_n_minus_1(Cu, u, n)
            assert np.linalg.norm(g - (g @ u) * u) < 3e-5
            agree += ttm.angle_deg(u, u_s) < 0.05
    assert total >= 55 and agree == total


def test_newton_ascent_halves_steps_that_fall():
    """A Newton step that lowers lambda is halved (at most twice) instead of
    ending the search.  Where the full-step search succeeds both take the same
    steps; where only the halving search succeeds, its answer is checked by
    plain evaluation: lambda rose from the start, and no point 0.5 or 2 degrees
    around the answer has a larger value (a local maximum of <C, u^n>)."""
    rng = np.random.default_rng(45)
    n = 6
    rescued = 0
    for _ in range(600):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        C = sym.monomials(v, n) + 0.5 * rng.standard_normal(28)
        Cu = C / ttm.score(C, n)
        w = np.cross(v, rng.standard_normal(3))
        u0 = np.cos(np.radians(25.0)) * v + np.sin(np.radians(25.0)) * w / np.linalg.norm(w)
        u_f, lam_f, ok_f = ttm.newton_ascent(Cu, n, u0, 5, 1e-5, halvings=0)
        u_h, lam_h, ok_h = ttm.newton_ascent(Cu, n, u0, 5, 1e-5)
        if ok_f:
            assert ok_h and np.array_equal(u_f, u_h) and lam_f == lam_h
            continue
        if not ok_h:
            continue
        rescued += 1
        assert lam_h >= sym.inner_power(Cu, u0, n) - 5e-6
        assert lam_h == pytest.approx(sym.inner_power(Cu, u_h, n), abs=1e-12)
        e1 = np.cross(u_h, rng.standard_normal(3))
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(u_h, e1)
        for deg in (0.5, 2.0):
            for k in range(64):
                ph = 2 * np.pi * k / 64
                p = np.cos(np.radians(deg)) * u_h + np.sin(np.radians(deg)) * (np.cos(ph) * e1 + np.sin(ph) * e2)
                assert sym.inner_power(Cu, p, n) <= lam_h + 1e-9
    assert rescued >= 5


# ---------------------------------------------------------------- field at single voxels
def test_field_at_equals_volume_field_and_guard():
    """field_at (w and C from one voxel's template window, what the full-size
    parity rests on) equals the whole-volume oracle (local_normalization,
    tensor_field) at the same voxels, including voxels whose window is
    constant, where the variance guard gives w = 0 (Eq. norm_f)."""
    D, L, r, n = 30, 8, 3.5, 4
    rng = np.random.default_rng(19)
    f = rng.standard_normal((D, D, D))
    f[2:16, 3:17, 4:18] = 1.75                      # windows inside are constant after h*
    g = ttm.prefilter_volume(f)
    m = ttm.ball_mask(L, r)
    wm = ttm.local_normalization(g, m)
    T = ttm.tensor_template(ttm.normalize_template(ndi.gaussian_filter(rng.standard_normal((L, L, L)), 1.0), r),
                            synth.rotation_samples(2), n)
    C = ttm.tensor_field(g, wm, T)
    c = L // 2
    lo, hi = ttm.valid_range(D, L)
    pts = [(lo, lo, lo), (hi, hi, hi), (8, 9, 10), (7, 8, 9)] + \
          [tuple(int(v) for v in rng.integers(lo, hi + 1, 3)) for _ in range(12)]
    patches = ttm.patches_at(g, pts, L)
    w1, C1 = ttm.field_at(patches, m, T, ttm.volume_g2_mean(g))
    guard = 0
    for i, (z, y, x) in enumerate(pts):
        want_w = wm[z, y, x]
        want_C = C[:, z - c, y - c, x - c]
        if want_w == 0:
            guard += 1
            assert w1[i] == 0 and np.all(C1[i] == 0)
        else:
            assert w1[i] == pytest.approx(want_w, rel=1e-12)
            assert np.allclose(C1[i], want_C, rtol=1e-12, atol=1e-12 * np.abs(want_C).max())
    assert guard >= 2
    # the windows can also be filtered from f directly (replicated borders)
    patches_f = ttm.patches_at(None, pts, L, f=f)
    assert np.allclose(patches_f, patches, atol=1e-13)


# ---------------------------------------------------------------- quaternion form (d' = 4)
def _left_mul(g):
    """4 x 4 matrix of q -> g q (Hamilton product), g = (w, x, y, z)."""
    w, x, y, z = g
    return np.array([[w, -x, -y, -z], [x, w, -z, y], [y, z, w, -x], [z, -y, x, w]])


def test_quaternion_form_rank_one_and_degree_two():
    rng = np.random.default_rng(51)
    st = synth.start_vectors(dim=4).astype(np.float64)
    for n in (2, 4, 6):
        for _ in range(3):
            q = rng.standard_normal(4)
            q /= np.linalg.norm(q)
            lam0 = rng.uniform(0.5, 2.0)
            C = lam0 * sym.monomials(q, n)
            lam, u, *_ = ttm.orient_multistart(C, n, st)
            assert lam == pytest.approx(lam0, rel=1e-10)
            assert ttm.quat_angle_deg(u, q) < 1e-5 and u[0] >= 0
            assert ttm.score(C, n, 4) == pytest.approx(lam0)
    for _ in range(6):
        A = rng.standard_normal((4, 4))
        A = A + A.T
        C = sym.from_full(A, 2, 4)
        ev, evec = np.linalg.eigh(A)
        lam, u, *_ = ttm.orient_multistart(C, 2, st)
        assert lam == pytest.approx(ev[-1], rel=1e-10)
        assert ttm.angle_deg(u, evec[:, -1]) < 1e-5


def test_quaternion_orientation_follows_left_multiplication():
    """Rotating the copy by g maps the optimal quaternion q to g q: the tensor
    transforms with the orthogonal map L_g (P-4 for d' = 4)."""
    rng = np.random.default_rng(52)
    st = synth.start_vectors(count=32, dim=4).astype(np.float64)
    n = 4
    for _ in range(3):
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        C = 2.0 * sym.monomials(q, n) + 0.2 * rng.standard_normal(35)
        g = rng.standard_normal(4)
        g /= np.linalg.norm(g)
        Lg = _left_mul(g)
        assert np.allclose(Lg.T @ Lg, np.eye(4))
        lam, u, *_ = ttm.orient_multistart(C, n, st)
        lam2, u2, *_ = ttm.orient_multistart(sym.rotate(C, Lg, n), n, st)
        assert lam2 == pytest.approx(lam, rel=1e-9)
        assert ttm.quat_angle_deg(u2, Lg @ u) < 1e-4
        assert ttm.score(sym.rotate(C, Lg, n), n, 4) == pytest.approx(ttm.score(C, n, 4))


def test_quaternion_tensor_template_equivariance():
    """P-5 for d' = 4: T(c + G (p - c)) = L_g^{(x)n} T(p) for a cube rotation G
    with quaternion g, because Q is closed under left multiplication by g."""
    L, r, n = 11, 4.0, 2
    rng = np.random.default_rng(53)
    t = ndi.gaussian_filter(rng.standard_normal((L, L, L)), 1.0)
    tn = ttm.normalize_template(t, r)
    Q = synth.rotation_samples(2)
    T = ttm.tensor_template(tn, Q, n, dprime=4)
    c = L // 2
    idx = np.arange(L) - c
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    P = np.stack([xx, yy, zz], axis=-1)
    for g in synth.octahedral_quaternions()[1:7]:
        G = rot.quat_to_matrix(g)
        dst = np.rint(P @ G.T).astype(int) + c
        lhs = T[:, dst[..., 2], dst[..., 1], dst[..., 0]]
        Lg = _left_mul(g)
        rhs = np.stack([sym.rotate(T[:, z, y, x], Lg, n) for z in range(L) for y in range(L)
                        for x in range(L)], axis=1).reshape(T.shape)
        assert np.allclose(lhs, rhs, atol=1e-12)


def test_reference_maxima_quaternion_agree_with_multistart():
    rng = np.random.default_rng(54)
    n = 4
    st = synth.start_vectors(count=64, dim=4).astype(np.float64)
    for _ in range(3):
        C = rng.standard_normal(35)
        lam, u, *_ = ttm.orient_multistart(C, n, st)
        lr, ur, l2 = ttm.reference_maxima(C, n, grid=20000, dprime=4)
        assert lr >= lam - 1e-9
        if lr - lam < 1e-9:
            assert ttm.quat_angle_deg(u, ur) < 1e-3


# ---------------------------------------------------------------- TTM-ref (Alg. 3)
def _planted_copy():
    w = synth.make_tomogram("ref", (36, 36, 36), L=12, n_blobs=3, n_copies=1, min_sep=12,
                            mask_radius=5.0, degree=4, seed=5, snr=None, wedge=False,
                            copy_amplitude=50.0)
    g = ttm.prefilter_volume(w.volume)
    wm = ttm.local_normalization(g, ttm.ball_mask(12, 5.0))
    tn = ttm.normalize_template(w.template, 5.0)
    return w, g, wm, tn


def test_sphere_offsets():
    o = ttm.sphere_offsets(3.0)
    assert len(o) == 123 and np.array_equal(o[0], [0, 0, 0])
    assert np.all(np.sum(o ** 2, axis=1) <= 9)
    rest = [tuple(v) for v in o[1:]]
    assert rest == sorted(rest) and len(set(rest)) == 122


def test_lncc_at_equals_rotation_sampled_tm():
    """Eq. lncc at one voxel (a window of g and t' rotated by trilinear
    pull-back) equals the whole-volume rotation-sampled TM of the oracle."""
    w, g, wm, tn = _planted_copy()
    rng = np.random.default_rng(61)
    qs = synth.random_quaternions(rng, 3)
    c = 6
    full = ttm.brute_force_tm(g, wm, tn, qs)
    for k, q in enumerate(qs):
        for _ in range(4):
            x = rng.integers(c, 36 - 12 + c + 1, 3)
            assert ttm.lncc_at(g, wm, tn, x, q) == pytest.approx(full[k, x[0] - c, x[1] - c, x[2] - c],
                                                                 rel=1e-12, abs=1e-14)


def _quat_of(R):
    """Unit quaternion of a rotation matrix (largest-component formula)."""
    qw = np.sqrt(max(0.0, 1 + np.trace(R))) / 2
    qx = np.copysign(np.sqrt(max(0.0, 1 + R[0, 0] - R[1, 1] - R[2, 2])) / 2, R[2, 1] - R[1, 2])
    qy = np.copysign(np.sqrt(max(0.0, 1 - R[0, 0] + R[1, 1] - R[2, 2])) / 2, R[0, 2] - R[2, 0])
    qz = np.copysign(np.sqrt(max(0.0, 1 - R[0, 0] - R[1, 1] + R[2, 2])) / 2, R[1, 0] - R[0, 1])
    return np.array([qw, qx, qy, qz])


def test_refine_returns_the_planted_centre_with_the_exact_rotation():
    """Alg. 3 with the planted copy's own rotation at every voxel: the LNCC at
    that rotation peaks at the planted centre, so a peak detected a few voxels
    off (inside r_s) is moved onto it; the peak's own values are reported too."""
    w, g, wm, tn = _planted_copy()
    qt = _quat_of(w.rotations[0])
    assert np.allclose(rot.quat_to_matrix(qt), w.rotations[0], atol=1e-12)
    ctr = w.centres[0]
    peaks = np.array([ctr + np.array([1, -1, 1]), ctr + np.array([0, 2, -1])])
    res = ttm.refine_positions(g, wm, tn, lambda x: None, lambda C: qt, peaks, 3.0)
    for (pos, q, c, q0, c0), p in zip(res, peaks):
        assert np.array_equal(pos, ctr)
        assert c == pytest.approx(ttm.lncc_at(g, wm, tn, ctr, qt), rel=1e-12)
        assert c0 == pytest.approx(ttm.lncc_at(g, wm, tn, p, qt), rel=1e-12) and c > c0 > 0


def test_refine_keeps_the_peak_on_ties():
    """Only a strictly larger LNCC moves the position (x~ starts at x^i): with
    w = 0 every LNCC is 0 and the peak stays."""
    w, g, wm, tn = _planted_copy()
    peaks = np.array([w.centres[0] + np.array([1, 1, 0])])
    res = ttm.refine_positions(g, np.zeros_like(wm), tn, lambda x: None,
                               lambda C: np.array([1.0, 0, 0, 0]), peaks, 3.0)
    assert np.array_equal(res[0][0], peaks[0]) and res[0][2] == 0.0


def test_certify_accepts_near_maxima_and_refuses_others():
    """The learned start's acceptance test: at a maximum the Newton step is
    zero; 10 degrees from a rank-one maximum a few Newton steps bring it within
    the step bound; at a minimum of <C, u^n> (the tangent Hessian is positive
    definite) nothing is certified."""
    rng = np.random.default_rng(71)
    n = 6
    for _ in range(4):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        C = sym.monomials(v, n)
        u, ok, step = ttm.certify(C, n, v)
        assert ok and step < 1e-12 and np.allclose(u, v)
        w = np.cross(v, rng.standard_normal(3))
        u0 = np.cos(np.radians(10.0)) * v + np.sin(np.radians(10.0)) * w / np.linalg.norm(w)
        u, ok, step = ttm.certify(C, n, u0)
        assert ok and step <= 1e-2 and ttm.angle_deg(u, v) < 1.0
        # -C has its minimum (for <C, u^n>: the maximum of -C's value) at v
        u, ok, step = ttm.certify(-C, n, v)
        assert not ok


def _axial_template(L):
    """Three blobs on the z axis, round across it: a template symmetric about z."""
    s = L / 24.0
    cz = s * np.array([[0, 0, -6.0], [0, 0, 1.0], [0, 0, 6.0]])
    return synth.BlobTemplate(L=L, centres=cz, axes=np.stack([np.eye(3)] * 3),
                              sigmas=s * np.array([[1.2, 1.2, 1.5], [2.2, 2.2, 1.2],
                                                   [0.9, 0.9, 0.9]]))


def _chiral_template(L):
    """Three unequal blobs on three different axes: no rotation maps it near itself."""
    s = L / 24.0
    c = s * np.array([[6.0, 0, 0], [0, 4.0, 0], [0, 0, -3.0]])
    return synth.BlobTemplate(L=L, centres=c, axes=np.stack([np.eye(3)] * 3),
                              sigmas=s * np.array([[1.0, 1.0, 1.0], [1.4, 1.4, 1.4],
                                                   [1.9, 1.9, 1.9]]))


@pytest.mark.parametrize("dprime", [3, 4])
def test_orientation_recovers_the_planted_rotation(dprime):
    """Ground truth from the renderer, not from the oracle: a copy rendered as
    t(R^T (p - x)) gives, at its centre, a field whose maximiser is R a in the
    axis form (for a template symmetric about a, the case that form is for) and
    the quaternion of R in the quaternion form (for a template that no rotation
    maps near itself).  A transposed rotation, a wrong monomial order or an
    axis in the wrong coordinate order lands tens of degrees away."""
    rng = np.random.default_rng(11)
    L, r, n, D = 24, 10.0, 4, 40
    tm = _axial_template(L) if dprime == 3 else _chiral_template(L)
    cen = np.array([[20, 19, 21]])
    m = ttm.ball_mask(L, r)
    tn = ttm.normalize_template(tm.volume(), r)
    T = ttm.tensor_template(tn, synth.rotation_samples(40), n, dprime=dprime)
    st = synth.start_vectors(count=64, dim=dprime).astype(np.float64)
    errs = []
    for R in synth.random_rotations(rng, 3):
        vol = synth.render_copies((D, D, D), tm, cen, R[None], scale=1.0)
        vol += 0.02 * rng.standard_normal(vol.shape)
        g = ttm.prefilter_volume(vol)
        Cv = ttm.field_at(ttm.patches_at(g, [cen[0]], L), m, T, ttm.volume_g2_mean(g))[1][0]
        u = ttm.orient_multistart(Cv, n, st)[1]
        u = u / np.linalg.norm(u)
        if dprime == 3:
            errs.append(np.degrees(np.arccos(min(1.0, abs(u @ R[:, 2])))))
        else:
            errs.append(np.degrees(2 * np.arccos(min(1.0, abs(u @ _quat_of(R))))))
    assert max(errs) < 8.0, errs


# ------------------------------------------------------- wedge-aware template
def test_wedge_filter_is_a_projection_that_removes_the_wedge():
    """W keeps a plane wave along x (k_z = 0), removes one along z (|k_z| > 0 =
    tan * |k_x|), keeps the mean, and is an orthogonal projection: W W = W and
    <W a, b> = <a, W b> (Parseval on the kept coefficients)."""
    P = 16
    keep = ttm.wedge_keep(P, 60.0)
    z, y, x = np.meshgrid(*[np.arange(P)] * 3, indexing="ij")

    def W(v):
        return np.fft.irfftn(np.fft.rfftn(v) * keep, s=(P, P, P), axes=(0, 1, 2))

    along_x = np.cos(2 * np.pi * 3 * x / P)
    along_z = np.cos(2 * np.pi * 2 * z / P)
    assert np.allclose(W(along_x), along_x, atol=1e-12)
    assert np.allclose(W(along_z), 0.0, atol=1e-12)
    assert np.allclose(W(np.full((P, P, P), 2.5)), 2.5, atol=1e-12)
    # |k_z| = 1, |k_x| = 1: kept at 60 degrees (tan 60 > 1), dropped at 30 degrees
    diag = np.cos(2 * np.pi * (x + z) / P)
    assert np.allclose(W(diag), diag, atol=1e-12)
    assert np.allclose(np.fft.irfftn(np.fft.rfftn(diag) * ttm.wedge_keep(P, 30.0), s=(P,) * 3,
                                     axes=(0, 1, 2)), 0.0,
                       atol=1e-12)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, P, P, P))
    assert np.allclose(W(W(a)), W(a), atol=1e-12)
    assert abs(np.sum(W(a) * b) - np.sum(a * W(b))) < 1e-9


def test_wedge_template_without_wedge_on_grid_rotations_is_alg1():
    """With W = I and the 24 grid-preserving rotations (no interpolation), each
    rotated t' is a permutation of t' inside the ball mask, already normalised,
    so the wedge-aware template equals Alg. 1's."""
    L, r, n = 13, 4.0, 4
    rng = np.random.default_rng(12)
    tn = ttm.normalize_template(ndi.gaussian_filter(rng.standard_normal((L, L, L)), 1.0), r)
    Q = synth.octahedral_quaternions()
    for dprime in (3, 4):
        T0 = ttm.tensor_template(tn, Q, n, dprime=dprime)
        T1 = ttm.tensor_template_wedge(tn, Q, n, r, None, 16, dprime=dprime)
        assert np.allclose(T0, T1, atol=1e-12)


def test_wedge_template_normalised_and_equivariant_under_wedge_symmetries():
    """The half turns G about x, y and z map the wedge onto itself and the
    rotation set onto itself, so the wedge-aware template is equivariant as
    Alg. 1's is: T(c + G (p - c)) = G^{(x)n} . T(p) (on the periodic padded box
    a half turn about c is the map x -> 2c - x mod P, which commutes with W).
    A rotation that does not map the wedge onto itself breaks it.
    Every rotated, filtered template has zero mean and unit norm on the mask."""
    L, r, n, P = 13, 4.0, 4, 16
    rng = np.random.default_rng(13)
    tn = ttm.normalize_template(ndi.gaussian_filter(rng.standard_normal((L, L, L)), 1.0), r)
    Q = synth.rotation_samples(1)
    m = ttm.ball_mask(L, r)
    T = ttm.tensor_template_wedge(tn, Q, n, r, 60.0, P)
    c = L // 2
    idx = np.arange(L) - c
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    Pts = np.stack([xx, yy, zz], axis=-1)
    for G in (np.diag([1.0, -1.0, -1.0]), np.diag([-1.0, 1.0, -1.0]), np.diag([-1.0, -1.0, 1.0])):
        dst = np.rint(Pts @ G.T).astype(int) + c
        lhs = T[:, dst[..., 2], dst[..., 1], dst[..., 0]]
        rhs = np.stack([sym.rotate(T[:, z, y, x], G, n) for z in range(L) for y in range(L)
                        for x in range(L)], axis=1).reshape(T.shape)
        assert np.allclose(lhs, rhs, atol=1e-10), np.abs(lhs - rhs).max()
    # a quarter turn about z does not preserve the wedge: the identity fails
    G = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    dst = np.rint(Pts @ G.T).astype(int) + c
    lhs = T[:, dst[..., 2], dst[..., 1], dst[..., 0]]
    rhs = np.stack([sym.rotate(T[:, z, y, x], G, n) for z in range(L) for y in range(L)
                    for x in range(L)], axis=1).reshape(T.shape)
    assert np.abs(lhs - rhs).max() > 1e-3
    keep = ttm.wedge_keep(P, 60.0)
    box = np.zeros((P, P, P))
    box[:L, :L, :L] = ttm.rotate_template(tn, ttm.quat_to_matrix(Q[5]))
    f = np.fft.irfftn(np.fft.rfftn(box) * keep, s=(P,) * 3, axes=(0, 1, 2))[:L, :L, :L]
    f = ttm.mask_normalize(f, m)
    assert abs(f.sum()) < 1e-10 and abs(np.sum(f * f) - 1.0) < 1e-10
