"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes are chosen so the oracle finishes in seconds while the GPU path still
runs several FFT tiles with ragged tails.  Tolerances:
* FFT: normwise relative error <= 2e-6 (FP32 transform of unit-variance data);
* scores: |c_gpu - c_orc| <= 1e-4 max(c_orc(x), median c_orc);
* field: ||dC(x)||_F <= 1e-4 max(c_orc(x), median c_orc);
* orientation: <= 1 degree at voxels whose best local maximum beats every
  other one (> 5 degrees away) by more than 1e-4 c; lambda within the score
  tolerance;
* peaks: bit-exact (positions and float values) on maps both sides read from
  the same input, and on full passes where the peak margins are clear.
"""
import math

import numpy as np
import pytest

import synth
from oracle import sym, ttm as orc
from tests.gpu_common import classify_orientation, rel_err, require_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    require_gpu()
    from paper_2408_02398_amd import ttm
    return ttm


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64) if t.dtype != torch.float64 else t.cpu().numpy()


# ------------------------------------------------------------------ FFT
@pytest.mark.parametrize("N", [32, 64, 96, 128, 160, 192, 256])
def test_fft_r2c_matches_numpy(T, ctx, N):
    print(f"[fft r2c N={N}]", flush=True)
    x = np.random.default_rng(N).standard_normal((N, N, N)).astype(np.float32)
    spec = host(T.fft3d_r2c(ctx, cuda(x)))
    got = spec[..., 0] + 1j * spec[..., 1]                     # [kz][kx][ky]
    want = np.fft.rfftn(x.astype(np.float64)).transpose(0, 2, 1)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 2e-6


@pytest.mark.parametrize("N", [32, 96])
def test_fft_small_direct_dft(T, ctx, N):
    """The forward transform against the DFT written out (no FFT library),
    for a power of two and for a mixed-radix edge (96 = 6 * 4 * 4)."""
    x = np.random.default_rng(5).standard_normal((N, N, N)).astype(np.float32)
    n = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(n, n) / N)              # DFT matrix, by definition
    want = np.einsum("az,by,cx,zyx->abc", W, W, W[: N // 2 + 1], x.astype(np.float64), optimize=True)
    spec = host(T.fft3d_r2c(ctx, cuda(x)))
    got = (spec[..., 0] + 1j * spec[..., 1]).transpose(0, 2, 1)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 2e-6


@pytest.mark.parametrize("N,L", [(32, 16), (64, 23), (96, 24), (160, 40), (192, 33), (256, 40)])
def test_template_planes_match_dft(T, ctx, N, L):
    """Template arrays of ttm_template_spectra: the K fields and the mask placed at
    the origin of a zero N^3 tile, transformed along x (half spectrum) and y, their
    L nonzero z planes kept, layout [z][kx][ky] (the z transform is left to the
    correlation, Alg. 2)."""
    print(f"[template planes N={N} L={L}]", flush=True)
    r = 0.4 * L
    d = T.make_desc(2, L, r)
    K = 6
    Tf = np.random.default_rng(N + L).standard_normal((K, L, L, L)).astype(np.float32)
    spec = host(T.template_spectra(ctx, d, cuda(Tf.reshape(K, -1)), N))
    assert spec.shape == (K + 1, L, N // 2 + 1, N, 2)
    assert T.template_spectrum_elems(N, L) == L * (N // 2 + 1) * N
    got = spec[..., 0] + 1j * spec[..., 1]
    fields = np.concatenate([Tf.astype(np.float64), orc.ball_mask(L, r)[None].astype(np.float64)])
    pad = np.zeros((K + 1, L, N, N))
    pad[:, :, :L, :L] = fields
    want = np.fft.fft(np.fft.rfft(pad, axis=3), axis=2).transpose(0, 1, 3, 2)   # [a][z][kx][ky]
    for a in range(K + 1):
        assert np.linalg.norm(got[a] - want[a]) / np.linalg.norm(want[a]) < 2e-6, a


@pytest.mark.parametrize("N", [32, 64, 96, 160, 192, 256])
def test_fft_roundtrip(T, ctx, N):
    x = np.random.default_rng(N + 1).standard_normal((N, N, N)).astype(np.float32)
    spec = T.fft3d_r2c(ctx, cuda(x))
    y = host(T.fft3d_c2r(ctx, spec, 1.0 / N ** 3))
    assert rel_err(y, x) < 2e-6


# ------------------------------------------------------------------ pipeline pieces
@pytest.fixture(scope="module")
def small():
    """A ragged multi-tile case: 50 x 61 x 72 volume, L = 12, FFT tiles of 32 (step 21)."""
    w = synth.make_tomogram("ragged", (50, 61, 72), L=12, n_blobs=3, n_copies=4, min_sep=12,
                            mask_radius=5.0, degree=4, seed=17, snr=None, wedge=False,
                            copy_amplitude=2.0)
    n, L, r = 4, 12, 5.0
    Q = synth.rotation_samples(10)
    tn = orc.normalize_template(w.template, r)
    Tt = orc.tensor_template(tn, Q, n)
    g = orc.prefilter_volume(w.volume)
    m = orc.ball_mask(L, r)
    wmap = orc.local_normalization(g, m)
    C = orc.tensor_field(g, wmap, Tt)
    return dict(w=w, n=n, L=L, r=r, Q=Q, tn=tn, Tt=Tt, g=g, wmap=wmap, C=C,
                score=orc.score(C, n))


def test_build_tensor_matches_oracle(T, ctx, small):
    d = T.make_desc(small["n"], small["L"], small["r"])
    Tg, tng = T.build_tensor(ctx, d, cuda(small["w"].template), cuda(small["Q"]))
    assert rel_err(host(tng), small["tn"]) < 2e-6
    err = np.linalg.norm(host(Tg) - small["Tt"]) / np.linalg.norm(small["Tt"])
    assert err < 1e-5


def test_normalize_matches_oracle(T, ctx, small):
    d = T.make_desc(small["n"], small["L"], small["r"])
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), 32)
    vol = cuda(small["w"].volume)
    g, w, stats = T.normalize(ctx, d, vol, spec, 32)
    st = stats.cpu().numpy()
    assert st[0] == pytest.approx(np.mean(small["g"]), rel=1e-6, abs=1e-9)
    assert st[1] == pytest.approx(np.mean(small["g"] ** 2), rel=1e-6)
    assert rel_err(host(g), small["g"]) < 1e-6
    wg, wo = host(w), small["wmap"]
    assert np.all(wg[wo == 0] == 0)
    nz = wo > 0
    assert np.max(np.abs(wg[nz] - wo[nz]) / wo[nz]) < 1e-4


@pytest.mark.parametrize("a", [2.0 ** -14, 2.0 ** 13])
def test_normalize_at_intensity_scales(T, ctx, small, a):
    """w of the tomogram scaled by a is the oracle's w / a (Eq. norm_f; the oracle's
    scale invariance is pinned on the CPU).  a is a power of two, so the scaled input
    is exact: the local sums must keep their relative precision at any intensity scale
    (a pass that mixes the first and second sums in one FP32 transform would not)."""
    d = T.make_desc(small["n"], small["L"], small["r"])
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), 32)
    _, w, _ = T.normalize(ctx, d, cuda(small["w"].volume * np.float32(a)), spec, 32)
    wg, wo = host(w) * a, small["wmap"]
    assert np.all(wg[wo == 0] == 0)
    nz = wo > 0
    assert np.max(np.abs(wg[nz] - wo[nz]) / wo[nz]) < 1e-4


def test_prefilter_and_box_normalisation_reproduce_normalize(T, ctx, small):
    """ttm_prefilter + ttm_normalize_box over the tile boxes == ttm_normalize, bit for bit,
    and a box that is not step-aligned still matches to FP32 rounding."""
    d = T.make_desc(small["n"], small["L"], small["r"])
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), 32)
    vol = cuda(small["w"].volume)
    g0, w0, s0 = T.normalize(ctx, d, vol, spec, 32)
    g1, w1, s1 = T.prefilter(ctx, d, vol)
    assert torch.equal(g0, g1) and torch.equal(s0, s1)
    assert torch.count_nonzero(w1).item() == 0
    for lo, size in T.tile_boxes(tuple(vol.shape), small["L"], 32):
        T.normalize_box(ctx, d, g1, s1, spec, 32, lo, size, w1)
    torch.cuda.synchronize()
    assert torch.equal(w0, w1)
    lo, hi = T.valid_bounds(tuple(vol.shape), small["L"])
    w2 = torch.zeros_like(w1)
    box_lo = (lo[0] + 3, lo[1] + 5, lo[2] + 1)
    box = (min(20, hi[0] - box_lo[0] + 1), min(9, hi[1] - box_lo[1] + 1), min(25, hi[2] - box_lo[2] + 1))
    T.normalize_box(ctx, d, g1, s1, spec, 32, box_lo, box, w2)
    sl = tuple(slice(a, a + b) for a, b in zip(box_lo, box))
    a, b = host(w2)[sl], host(w0)[sl]
    assert np.max(np.abs(a - b) / np.maximum(b, 1e-30)) < 1e-4
    assert np.count_nonzero(host(w2)) == np.count_nonzero(a)
    from paper_2408_02398_amd._lib import TTMError
    with pytest.raises(TTMError):
        T.normalize_box(ctx, d, g1, s1, spec, 32, (0, 0, 0), (4, 4, 4), w2)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_correlate_and_score_match_oracle(T, ctx, small, dtype):
    n, L = small["n"], small["L"]
    d = T.make_desc(n, L, small["r"])
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), 32)
    g, w, stats = T.normalize(ctx, d, cuda(small["w"].volume), spec, 32)
    lo, hi = T.valid_bounds(small["w"].volume.shape, L)
    size = tuple(h - l + 1 for l, h in zip(lo, hi))
    Cg = T.correlate(ctx, d, g, w, stats, spec, 32, lo, size, dtype=dtype)
    Cg_h = host(Cg)
    Co = small["C"]
    cs = small["score"]
    floor = np.maximum(cs, np.median(cs))
    dC = np.sqrt(np.tensordot(sym.weights(n, 3), (Cg_h - Co) ** 2, axes=(0, 0)))
    tol = 1e-4 if dtype == torch.float32 else 1e-2
    assert np.max(dC / floor) < tol
    score, _, _ = T.extract(ctx, d, Cg, orient=False)
    sg = host(score)
    assert np.max(np.abs(sg - cs) / floor) < tol


@pytest.mark.parametrize("N,L", [(64, 48), (96, 40), (128, 64), (160, 48), (192, 64), (256, 64),
                                 (512, 64)])
def test_large_templates_sampled(T, ctx, N, L):
    """The largest templates (L = 64) and ones whose z planes need several
    slots per thread in the Z-inverse pass (8 at N = 64 and 128, 4 at N = 256,
    2 at N = 512): w and C on one full tile, checked at sampled voxels against
    the FP64 oracle's direct sums (Eq. norm_f, Eq. tcc)."""
    print(f"[large template N={N} L={L}]", flush=True)
    n, K, r = 2, 6, 0.4 * L
    d = T.make_desc(n, L, r)
    rng = np.random.default_rng(N + L)
    D = L + 40
    vol = rng.standard_normal((D, D, D)).astype(np.float32)
    Tf = (rng.standard_normal((K, L, L, L)) / L ** 1.5).astype(np.float32)
    spec = T.template_spectra(ctx, d, cuda(Tf.reshape(K, -1)), N)
    g, w, stats = T.normalize(ctx, d, cuda(vol), spec, N)
    lo, hi = T.valid_bounds(vol.shape, L)
    size = tuple(h - l + 1 for l, h in zip(lo, hi))
    Cg = host(T.correlate(ctx, d, g, w, stats, spec, N, lo, size))
    wg = host(w)
    pts = [tuple(lo), tuple(hi)] + [tuple(int(rng.integers(a, b + 1)) for a, b in zip(lo, hi))
                                    for _ in range(4)]
    c = L // 2
    patches = np.stack([orc.prefilter_box(vol, (z - c, y - c, x - c), (z - c + L, y - c + L, x - c + L))
                        for z, y, x in pts])
    g2 = float(np.mean(orc.prefilter_volume(vol) ** 2))
    wo, Co = orc.field_at(patches, orc.ball_mask(L, r), Tf.astype(np.float64), g2)
    del patches
    assert np.all(wo > 0)
    wgs = np.array([wg[p] for p in pts])
    assert np.max(np.abs(wgs - wo) / wo) < 1e-4
    Cgs = np.stack([Cg[:, z - lo[0], y - lo[1], x - lo[2]] for z, y, x in pts])
    so = orc.score(Co.T, n)
    floor = np.maximum(so, np.median(so))
    dC = np.sqrt(np.sum(sym.weights(n, 3) * (Cgs - Co) ** 2, axis=1))
    assert np.max(dC / floor) < 1e-4


def test_correlate_sub_box_and_single_voxel(T, ctx, small):
    n, L = small["n"], small["L"]
    d = T.make_desc(n, L, small["r"])
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), 32)
    g, w, stats = T.normalize(ctx, d, cuda(small["w"].volume), spec, 32)
    c = L // 2
    for lo, size in [((c + 3, c + 5, c + 7), (30, 9, 44)), ((c, c, c), (1, 1, 1)),
                     ((38, 49, 60), (1, 1, 1))]:
        Cg = host(T.correlate(ctx, d, g, w, stats, spec, 32, lo, size))
        Co = small["C"][:, lo[0] - c:lo[0] - c + size[0], lo[1] - c:lo[1] - c + size[1],
                        lo[2] - c:lo[2] - c + size[2]]
        cs = orc.score(Co, n)
        floor = np.maximum(cs, np.median(small["score"]))
        dC = np.sqrt(np.tensordot(sym.weights(n, 3), (Cg - Co) ** 2, axes=(0, 0)))
        assert np.max(dC / floor) < 1e-4


def test_orientation_matches_oracle(T, ctx, small):
    """Every one of 160 sampled voxels: the GPU's (lambda, u) agrees with the
    oracle's converged multistart answer (within 1 degree, lambda within the
    score tolerance) or is a near-optimal maximiser of the FP64 function
    (flat or tied maxima); none is left unclassified."""
    n = small["n"]
    d = T.make_desc(n, small["L"], small["r"])
    Co = small["C"]
    K = Co.shape[0]
    rng = np.random.default_rng(3)
    flat = Co.reshape(K, -1)
    idx = rng.choice(flat.shape[1], 160, replace=False)
    Cs = np.ascontiguousarray(flat[:, idx]).reshape(K, 1, 1, -1)
    starts = synth.start_vectors()
    score, lam, u = T.extract(ctx, d, cuda(Cs), starts=cuda(starts), max_iter=500, tol=1e-5)
    lg, ug = host(lam).ravel(), host(u).reshape(-1, 3)
    med = np.median(orc.score(Co, n))
    counts = {"agree": 0, "near": 0}
    for j, i in enumerate(idx):
        v = flat[:, i]
        lam_o, u_o, *_ = orc.orient_multistart(v, n, starts.astype(np.float64))
        cls, info = classify_orientation(v, n, lg[j], ug[j], lam_o, u_o, max(orc.score(v, n), med))
        assert cls is not None, (j, info)
        counts[cls] += 1
    print(f"[orientation 160 voxels] {counts}", flush=True)
    assert counts["agree"] >= 0.8 * len(idx)


def test_orientation_rank_one_and_zero(T, ctx):
    n = 6
    d = T.make_desc(n, 16, 7.0)
    rng = np.random.default_rng(9)
    vs = rng.standard_normal((64, 3))
    vs /= np.linalg.norm(vs, axis=1, keepdims=True)
    lam0 = rng.uniform(0.5, 2.0, 64)
    C = (lam0[:, None] * sym.monomials(vs, n)).T.reshape(28, 1, 1, 64).copy()
    C[:, 0, 0, 0] = 0.0                                          # zero tensor
    score, lam, u = T.extract(ctx, d, cuda(C), starts=cuda(synth.start_vectors()))
    lg, ug, sg = host(lam).ravel(), host(u).reshape(-1, 3), host(score).ravel()
    assert lg[0] == 0 and np.all(ug[0] == 0) and sg[0] == 0
    assert np.allclose(lg[1:], lam0[1:], rtol=1e-4)
    assert np.allclose(sg[1:], lam0[1:], rtol=1e-5)
    assert np.max(orc.angle_deg(ug[1:], vs[1:])) < 0.05
    # canonical sign: last non-zero coordinate positive
    assert np.all(ug[1:, 2] > 0)


# ------------------------------------------------------------------ peaks
@pytest.mark.parametrize("seed,shape,P,D", [(1, (20, 23, 26), 40, 3.0), (2, (40, 41, 42), 200, 5.5),
                                            (3, (9, 10, 11), 5000, 1.0),
                                            # P beyond what fits at distance D: every
                                            # candidate is walked
                                            (5, (40, 52, 60), 2000, 6.0),
                                            # rows wider than one 1024-column compaction
                                            # block, ragged row blocks in y
                                            (6, (6, 37, 1100), 300, 4.5)])
def test_find_peaks_bit_exact_on_shared_map(T, ctx, seed, shape, P, D):
    rng = np.random.default_rng(seed)
    s = np.round(rng.uniform(0, 1, shape), 3).astype(np.float32)   # many exact ties
    lo = (1, 2, 3)
    hi = (shape[0] - 2, shape[1] - 1, shape[2] - 4)
    P = min(P, 2000)
    pk, pv = T.find_peaks(ctx, cuda(s), lo, hi, P, D)
    pko, pvo = orc.find_peaks(s.astype(np.float64), lo, hi, P, D)
    assert np.array_equal(pk.cpu().numpy().astype(np.int64), pko)
    assert np.array_equal(pv.cpu().numpy(), pvo.astype(np.float32))


def test_peak_errors(T, ctx):
    from paper_2408_02398_amd._lib import TTMError
    s = cuda(np.zeros((8, 8, 8), np.float32))
    with pytest.raises(TTMError):
        T.find_peaks(ctx, s, (0, 0, 0), (8, 7, 7), 3, 1.0)      # region outside the map
    with pytest.raises(TTMError):
        T.find_peaks(ctx, s, (0, 0, 0), (7, 7, 7), 0, 1.0)      # top_p < 1


def test_boundary_errors(T, ctx, small):
    from paper_2408_02398_amd._lib import TTMError
    d = T.make_desc(4, 12, 5.0)
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), 32)
    g, w, stats = T.normalize(ctx, d, cuda(small["w"].volume), spec, 32)
    with pytest.raises(TTMError):   # box outside the valid region
        T.correlate(ctx, d, g, w, stats, spec, 32, (0, 6, 6), (2, 2, 2))
    bad = T.make_desc(3, 12, 5.0)  # odd degree
    with pytest.raises(TTMError):
        T.correlate(ctx, bad, g, w, stats, spec, 32, (6, 6, 6), (2, 2, 2))
    big = T.make_desc(4, 40, 17.0)
    with pytest.raises(TTMError):   # L > FFT edge
        T.template_spectra(ctx, big, cuda(np.zeros((15, 40, 40, 40), np.float32)), 32)
    with pytest.raises(TTMError):
        T.fft3d_r2c(ctx, cuda(np.zeros((48, 48, 48), np.float32)))   # unsupported edge


# ------------------------------------------------------------------ full pass, 64^3, n = 4
def test_full_pass_64cube(T, ctx):
    print("[full pass 64^3 n=4]", flush=True)
    w = synth.make_config("c1_64cube_n4")
    n, L, r = 4, 16, 7.0
    Q = synth.rotation_samples(50)
    d = T.make_desc(n, L, r)
    Tg, _ = T.build_tensor(ctx, d, cuda(w.template), cuda(Q))
    spec = T.template_spectra(ctx, d, Tg, 64)
    starts = cuda(synth.start_vectors())
    eng = T.Engine(ctx, d, spec, 64, w.volume.shape, starts)
    res = eng.run(cuda(w.volume), top_p=5)
    # oracle
    tn = orc.normalize_template(w.template, r)
    Tt = orc.tensor_template(tn, Q, n)
    g = orc.prefilter_volume(w.volume)
    wm = orc.local_normalization(g, orc.ball_mask(L, r))
    C = orc.tensor_field(g, wm, Tt)
    cs = orc.score(C, n)
    lo, hi = T.valid_bounds(w.volume.shape, L)
    sg = host(res.score)[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
    floor = np.maximum(cs, np.median(cs))
    assert np.max(np.abs(sg - cs) / floor) < 1e-4
    full = np.zeros(w.volume.shape)
    full[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = cs
    pko, pvo = orc.find_peaks(full, lo, hi, 5, 2 * r)
    pk = res.peaks.cpu().numpy().astype(np.int64)
    assert np.array_equal(pk, pko)
    # orientation at every peak: agreement with the oracle's converged answer,
    # or a near-optimal maximiser of the FP64 function (flat or tied maxima)
    ug, lgm = host(res.direction), host(res.lam)
    counts = {"agree": 0, "near": 0}
    for p in pko:
        v = C[:, p[0] - lo[0], p[1] - lo[1], p[2] - lo[2]]
        lam_o, u_o, *_ = orc.orient_multistart(v, n, synth.start_vectors().astype(np.float64))
        cls, info = classify_orientation(v, n, lgm[tuple(p)], ug[tuple(p)], lam_o, u_o,
                                         max(orc.score(v, n), np.median(cs)))
        assert cls is not None, (p, info)
        counts[cls] += 1
    assert sum(counts.values()) == 5


# ------------------------------------------------------------------ guard and quaternion form
def test_constant_tomogram_gives_zero_weight(T, ctx):
    """A constant tomogram has zero local variance everywhere: the guard of
    Eq. norm_f gives w = 0, and with it C = 0 and a zero score (no division by
    a vanishing variance)."""
    n, L, r = 4, 12, 5.0
    d = T.make_desc(n, L, r)
    K = sym.n_components(n, 3)
    Tf = np.random.default_rng(1).standard_normal((K, L, L, L)).astype(np.float32)
    spec = T.template_spectra(ctx, d, cuda(Tf.reshape(K, -1)), 32)
    vol = cuda(np.full((40, 37, 45), 2.5, np.float32))
    g, w, stats = T.normalize(ctx, d, vol, spec, 32)
    assert torch.count_nonzero(w).item() == 0
    lo, hi = T.valid_bounds(tuple(vol.shape), L)
    size = tuple(h - l + 1 for l, h in zip(lo, hi))
    Cg = T.correlate(ctx, d, g, w, stats, spec, 32, lo, size)
    assert torch.count_nonzero(Cg).item() == 0
    score, lam, u = T.extract(ctx, d, Cg, starts=cuda(synth.start_vectors()))
    assert torch.count_nonzero(score).item() == 0 and torch.count_nonzero(lam).item() == 0


def test_quaternion_form_tensor_field_and_score(T, ctx, small):
    """d' = 4 (the paper's quaternion form, K = 35 at n = 4): the tensor template
    (Alg. 1 with v_q = q), the tensor field (Alg. 2) and the Frobenius score
    against the oracle on the ragged multi-tile case."""
    print("[quaternion form n=4]", flush=True)
    n, L, r = 4, small["L"], small["r"]
    d = T.make_desc(n, L, r, dprime=4)
    K = sym.n_components(n, 4)
    assert T.n_components(n, 4) == K == 35
    Tg, _ = T.build_tensor(ctx, d, cuda(small["w"].template), cuda(small["Q"]))
    T4 = orc.tensor_template(small["tn"], small["Q"], n, dprime=4)
    assert np.linalg.norm(host(Tg) - T4) / np.linalg.norm(T4) < 1e-5
    spec = T.template_spectra(ctx, d, Tg, 32)
    g, w, stats = T.normalize(ctx, d, cuda(small["w"].volume), spec, 32)
    lo, hi = T.valid_bounds(small["w"].volume.shape, L)
    size = tuple(h - l + 1 for l, h in zip(lo, hi))
    Cg = T.correlate(ctx, d, g, w, stats, spec, 32, lo, size)
    Co = orc.tensor_field(small["g"], small["wmap"], T4)
    cs = orc.score(Co, n, 4)
    floor = np.maximum(cs, np.median(cs))
    dC = np.sqrt(np.tensordot(sym.weights(n, 4), (host(Cg) - Co) ** 2, axes=(0, 0)))
    assert np.max(dC / floor) < 1e-4
    score, _, _ = T.extract(ctx, d, Cg, orient=False)
    assert np.max(np.abs(host(score) - cs) / floor) < 1e-4


@pytest.mark.parametrize("n,n_vox", [(4, 120), (6, 48)])
def test_quaternion_orientation_matches_oracle(T, ctx, small, n, n_vox):
    """d' = 4 orientation (Sec. 3.1 on S^3, quaternions; K = 35 at n = 4, 84 at
    n = 6): rank-one tensors lambda0 q^n give back (lambda0, +-q) with w >= 0, a
    zero tensor gives 0, and at sampled voxels of the d' = 4 field every answer
    agrees with the oracle's converged multistart answer (rotation distance
    2 arccos|q1.q2| < 1 degree) or is a near-optimal maximiser of the FP64
    function."""
    print(f"[quaternion orientation n={n}]", flush=True)
    L, r = small["L"], small["r"]
    d = T.make_desc(n, L, r, dprime=4)
    K = T.n_components(n, 4)
    starts = synth.start_vectors(count=32, dim=4)
    rng = np.random.default_rng(21)
    qs = rng.standard_normal((64, 4))
    qs /= np.linalg.norm(qs, axis=1, keepdims=True)
    lam0 = rng.uniform(0.5, 2.0, 64)
    C = (lam0[:, None] * sym.monomials(qs, n)).T.reshape(K, 1, 1, 64).copy()
    C[:, 0, 0, 0] = 0.0
    score, lam, u = T.extract(ctx, d, cuda(C), starts=cuda(starts))
    lg, ug, sg = host(lam).ravel(), host(u).reshape(-1, 4), host(score).ravel()
    assert lg[0] == 0 and np.all(ug[0] == 0) and sg[0] == 0
    assert np.allclose(lg[1:], lam0[1:], rtol=1e-4)
    assert np.allclose(sg[1:], lam0[1:], rtol=1e-5)
    assert np.max(orc.quat_angle_deg(ug[1:], qs[1:])) < 0.05
    assert np.all(ug[1:, 0] >= 0)
    # sampled voxels of the d' = 4 field of the ragged case
    T4 = orc.tensor_template(small["tn"], small["Q"], n, dprime=4)
    Co = orc.tensor_field(small["g"], small["wmap"], T4)
    flat = Co.reshape(K, -1)
    idx = rng.choice(flat.shape[1], n_vox, replace=False)
    Cs = np.ascontiguousarray(flat[:, idx]).reshape(K, 1, 1, -1)
    _, lam, u = T.extract(ctx, d, cuda(Cs), starts=cuda(starts))
    lg, ug = host(lam).ravel(), host(u).reshape(-1, 4)
    med = np.median(orc.score(Co, n, 4))
    counts = {"agree": 0, "near": 0}
    for j, i in enumerate(idx):
        v = flat[:, i]
        lam_o, u_o, *_ = orc.orient_multistart(v, n, starts.astype(np.float64))
        cls, info = classify_orientation(v, n, lg[j], ug[j], lam_o, u_o, max(orc.score(v, n, 4), med))
        assert cls is not None, (j, info)
        counts[cls] += 1
    print(f"[quaternion orientation n={n}, {n_vox} voxels] {counts}", flush=True)
    assert counts["agree"] >= 0.8 * len(idx)


@pytest.mark.parametrize("L,dprime", [(13, 3), (12, 4)])
def test_wedge_tensor_template_matches_oracle(T, ctx, L, dprime):
    """ttm_build_tensor_wedge against the oracle's wedge-aware Alg. 1 (each
    rotated t' filtered by the +-60 degree missing wedge on its box padded to
    32^3, renormalised over the mask, then weighted by v_q^n): normwise 1e-5."""
    print(f"[wedge template L={L} d'={dprime}]", flush=True)
    n, r = 4, 4.5
    rng = np.random.default_rng(30 + L)
    t = rng.standard_normal((L, L, L)).astype(np.float32)
    Q = synth.rotation_samples(2)
    d = T.make_desc(n, L, r, dprime=dprime)
    Tg, tng = T.build_tensor(ctx, d, cuda(t), cuda(Q), wedge=60.0)
    tn = orc.normalize_template(t, r)
    assert rel_err(host(tng), tn) < 2e-6
    To = orc.tensor_template_wedge(tn, Q, n, r, 60.0, 32, dprime=dprime)
    err = np.linalg.norm(host(Tg) - To) / np.linalg.norm(To)
    print(f"[wedge template] normwise error {err:.2e}", flush=True)
    assert err < 1e-5
    # the wedge changes the template: Alg. 1 without it differs
    T0 = orc.tensor_template(tn, Q, n, dprime=dprime)
    assert np.linalg.norm(T0 - To) / np.linalg.norm(To) > 1e-2


def test_normalize_correlate_equals_the_two_calls(T, ctx, small):
    """ttm_normalize_correlate on one tile = ttm_normalize_box then
    ttm_correlate on it, bit for bit (the same forward transform of g)."""
    d = T.make_desc(small["n"], small["L"], small["r"])
    N = 32
    spec = T.template_spectra(ctx, d, cuda(small["Tt"]), N)
    vol = cuda(small["w"].volume)
    g, w, stats = T.normalize(ctx, d, vol, spec, N)
    step = N - small["L"] + 1
    lo, hi = T.valid_bounds(vol.shape, small["L"])
    for box_lo, size in (((lo[0], lo[1], lo[2]), (step, step, step)),
                         ((hi[0] - 6, hi[1] - 13, lo[2] + 3), (7, 14, 9))):
        w1 = torch.zeros_like(w)
        T.normalize_box(ctx, d, g, stats, spec, N, box_lo, size, w1)
        C1 = T.correlate(ctx, d, g, w1, stats, spec, N, box_lo, size)
        w2 = torch.zeros_like(w)
        C2 = T.normalize_correlate(ctx, d, g, stats, spec, N, box_lo, size, w2)
        torch.cuda.synchronize()
        assert torch.equal(w1, w2) and torch.equal(C1, C2)
    from paper_2408_02398_amd._lib import TTMError
    with pytest.raises(TTMError):
        T.normalize_correlate(ctx, d, g, stats, spec, N, (lo[0], lo[1], lo[2]), (step + 1, 4, 4),
                              torch.zeros_like(w))


@pytest.mark.parametrize("learned", [False, True])
def test_full_pass_is_deterministic(T, ctx, learned):
    """A full pass run twice, with the tile correlations overlapped on a side
    stream, gives the same w, score, lambda and direction maps and the same
    peaks, bit for bit: the pooled runs write each (voxel, start) result to its
    own slot whatever lane ran it, the reductions take the first maximum in
    start order, and the learned path's fallback list order does not reach any
    voxel's answer.  A 150 x 170 x 190 volume of the 256^3 workload's recipe on
    64^3 tiles (many tiles, ragged edges), degree 6."""
    from oracle import mlp as omlp
    from tests.gpu_common import oracle_trained_params
    print(f"[determinism learned={learned}]", flush=True)
    wl = synth.make_config("c2_256cube_n6", shape=(150, 170, 190), n_copies=20, min_sep=32)
    n, L, r = 6, 32, 14.0
    d = T.make_desc(n, L, r)
    Tg, _ = T.build_tensor(ctx, d, cuda(wl.template), cuda(synth.rotation_samples(10)))
    spec = T.template_spectra(ctx, d, Tg, 64)
    starts = cuda(synth.start_vectors())
    mlp = None
    if learned:
        mlp = T.MLP(ctx, d, cuda(omlp.pad_params(oracle_trained_params(13, n), 28)))
    eng = T.Engine(ctx, d, spec, 64, wl.volume.shape, starts, mlp=mlp, kappa=0.3)
    assert len(eng.boxes) > 8
    vol = cuda(wl.volume)
    outs = []
    for _ in range(2):
        res = eng.run(vol, top_p=20)
        torch.cuda.synchronize()
        outs.append([res.w.clone(), res.score.clone(), res.lam.clone(), res.direction.clone(),
                     res.peaks.clone(), res.peak_vals.clone()])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
