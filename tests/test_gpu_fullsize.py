"""Parity at the full workload sizes, in the launch configuration of the
benchmark: its FFT tile (512^3 for the 512 x 928 x 928 tomogram, one 256^3
transform for 256^3), tile correlations overlapped with extraction on a side
stream, Find Peaks over the whole volume.  The FP64 oracle cannot run a
whole 512 x 928 x 928 pass, so it computes sampled voxels one by one from the
raw tomogram (Eq. norm_f, Eq. tcc, Sec. 3.1 / 3.2): w, the score, lambda and
the orientation at the first peaks, at tile seams and at random valid voxels.
The tensor template uses 480 rotations on both sides to keep Alg. 1 in the
oracle within seconds; the rotation count does not change any kernel's work
per voxel.

Tolerances as in the small-size tests: w and the score within 1e-4 relative
(score relative to max(score, median score)).  Orientation: every sampled
voxel is classified against the oracle's converged answer (SS-HOPM to 1e-13,
then Newton to rounding level): it agrees (within 1 degree, lambda within the
score tolerance), or the GPU found a near-optimal maximiser of the FP64
function (a flat maximum or one of two tied maxima, whose position the FP32
field's rounding moves by more than a degree).  With the learned start the
network sees the GPU's FP32 field, not the oracle's FP64 one: at a voxel whose
start sits on a basin boundary, or whose fallback test is within rounding of
flipping, the GPU may take the other branch, whose answer it must then match
(a few such voxels only).  No voxel is left unclassified.
"""
import functools

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import sym, ttm as orc
from tests.gpu_common import classify_orientation, oracle_trained_params, require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


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


@functools.lru_cache(maxsize=2)
def workload(name):
    """Tomogram, rotations and the oracle's tensor template of one workload."""
    p = synth.CONFIGS[name]
    wl = synth.make_config(name)
    Q = synth.rotation_samples(20)
    Tt = orc.tensor_template(orc.normalize_template(wl.template, p["mask_radius"]), Q, p["degree"])
    return wl, Q, Tt


def sample_points(T, eng, shape, L, peaks, n_random, seed):
    lo, hi = T.valid_bounds(shape, L)
    rng = np.random.default_rng(seed)
    seams = []
    for (blo, size) in eng.boxes[:: max(1, len(eng.boxes) // 8)]:
        seams.append(tuple(blo))
        seams.append(tuple(a + s - 1 for a, s in zip(blo, size)))
    rnd = np.stack([rng.integers(a, b + 1, n_random) for a, b in zip(lo, hi)], 1)
    return np.concatenate([peaks, np.array(seams, dtype=np.int64), rnd]).astype(np.int64)


def oracle_field(vol, pts, L, r, Tt):
    """w and C at the sample voxels from FP64 windows of the prefiltered volume."""
    c = L // 2
    patches = np.stack([orc.prefilter_box(vol, (z - c, y - c, x - c), (z - c + L, y - c + L, x - c + L))
                        for z, y, x in pts])
    # mean of g^2 over the whole volume (enters only the variance guard), in slabs
    s2 = 0.0
    for z0 in range(0, vol.shape[0], 64):
        z1 = min(z0 + 64, vol.shape[0])
        g = orc.prefilter_box(vol, (z0, 0, 0), (z1, vol.shape[1], vol.shape[2]))
        s2 += float(np.sum(g * g))
    g2 = s2 / vol.size
    return orc.field_at(patches, orc.ball_mask(L, r), Tt, g2)


FFT_TILE = {"c2_256cube_n6": 256, "c3_512x928x928_n6": 512}


def learned_alternatives(Cv, n, pl, st, kappa):
    """(lambda, direction) of the learned path (Sec. 3.3 start, Sec. 3.1 ascent)
    from starts tilted 0.25 and 1 degree around the network's direction.  The
    GPU evaluates the network on its own FP32 field, whose rounding can move
    the start by about that much; where such a tilt crosses into another basin,
    each of these answers is one the method may give."""
    y, _ = omlp.forward(pl, omlp.features(Cv[None, :], n), bf16=True)
    u0 = y[0] / np.linalg.norm(y[0])
    a = np.cross(u0, [1.0, 0.0, 0.0])
    if np.linalg.norm(a) < 0.5:
        a = np.cross(u0, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(u0, a)
    out = []
    for deg in (0.25, 1.0):
        r = np.radians(deg)
        for k in range(6):
            ax = np.cos(np.pi * k / 3) * a + np.sin(np.pi * k / 3) * b
            lam, u, _ = omlp.orient_learned(Cv, n, pl, st, kappa, u0=np.cos(r) * u0 + np.sin(r) * ax)
            out.append((lam, u))
    return out


@pytest.mark.parametrize("name", ["c2_256cube_n6", "c3_512x928x928_n6"])
@pytest.mark.parametrize("start", ["multistart", "learned"])
def test_full_size_sampled_parity(T, ctx, name, start):
    say(f"[fullsize {name} {start}] generating")
    p = synth.CONFIGS[name]
    n, L, r = p["degree"], p["L"], p["mask_radius"]
    wl, Q, Tt = workload(name)
    d = T.make_desc(n, L, r)
    Tg, _ = T.build_tensor(ctx, d, cuda(wl.template), cuda(Q))
    spec = T.template_spectra(ctx, d, Tg, FFT_TILE[name])
    starts = synth.start_vectors()
    K = sym.n_components(n, 3)
    mlp, kappa, pl = None, 0.0, None
    if start == "learned":
        pl = oracle_trained_params(13, n)
        mlp, kappa = T.MLP(ctx, d, cuda(omlp.pad_params(pl, K))), 0.3
    eng = T.Engine(ctx, d, spec, FFT_TILE[name], wl.volume.shape, cuda(starts), mlp=mlp, kappa=kappa)
    say(f"[fullsize {name} {start}] GPU pass over {len(eng.boxes)} tiles")
    res = eng.run(cuda(wl.volume), top_p=50)
    torch.cuda.synchronize()
    peaks = res.peaks.cpu().numpy().astype(np.int64)
    pts = sample_points(T, eng, wl.volume.shape, L, peaks[:16], 80, 17)
    idx = (pts[:, 0], pts[:, 1], pts[:, 2])
    wg = res.w.cpu().numpy()[idx]
    sg = res.score.cpu().numpy()[idx]
    lg = res.lam.cpu().numpy()[idx]
    ug = res.direction.cpu().numpy()[idx]
    say(f"[fullsize {name} {start}] oracle on {len(pts)} voxels")
    wo, Co = oracle_field(wl.volume, pts, L, r, Tt)
    so = orc.score(Co.T, n)
    floor = np.maximum(so, np.median(so))
    assert np.all(wo > 0)
    assert np.max(np.abs(wg - wo) / wo) < 1e-4
    assert np.max(np.abs(sg - so) / floor) < 1e-4
    st = starts.astype(np.float64)
    counts = {"agree": 0, "near": 0, "alt": 0}
    for i in range(len(pts)):
        if i % 20 == 0:
            say(f"[fullsize {name} {start}] oracle orientation {i}/{len(pts)}")
        if start == "multistart":
            lam_o, u_o, *_ = orc.orient_multistart(Co[i], n, st)
            cls, info = classify_orientation(Co[i], n, lg[i], ug[i], lam_o, u_o, floor[i])
        else:
            lam_o, u_o, fell, det = omlp.orient_learned(Co[i], n, pl, st, kappa, detail=True)
            cls, info = classify_orientation(Co[i], n, lg[i], ug[i], lam_o, u_o, floor[i])
            if cls is None:
                # the other branch of a fallback test within rounding of flipping,
                # or a start within rounding of a basin boundary
                alts = [(det["lam_learned"], det["u_learned"]), orc.orient_multistart(Co[i], n, st)[:2]]
                alts += learned_alternatives(Co[i], n, pl, st, kappa)
                cls, info = classify_orientation(Co[i], n, lg[i], ug[i], lam_o, u_o, floor[i], alts)
        assert cls is not None, (i, pts[i], info)
        counts[cls] += 1
    say(f"[fullsize {name} {start}] orientation at {len(pts)} voxels: {counts}")
    assert counts["agree"] >= 0.8 * len(pts)
    assert counts["alt"] <= max(2, len(pts) // 20)
    # each of the first peaks is a local maximum of the oracle's score up to the
    # score tolerance (its face neighbours computed by the oracle)
    nb = np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
    pk16 = peaks[:16]
    npts = (pk16[:, None, :] + nb[None]).reshape(-1, 3)
    lo_v, hi_v = T.valid_bounds(wl.volume.shape, L)
    npts = np.clip(npts, lo_v, hi_v)
    _, Cn = oracle_field(wl.volume, npts, L, r, Tt)
    sn = orc.score(Cn.T, n).reshape(len(pk16), 6)
    so16 = so[:len(pk16)]
    for k in range(len(pk16)):
        for m_ in range(6):
            q = npts[6 * k + m_]
            # a neighbour that was a candidate (not excluded by an earlier peak)
            if k == 0 or np.min(np.sum((pk16[:k] - q) ** 2, axis=1)) >= (2 * r) ** 2:
                assert so16[k] >= sn[k, m_] - 2e-4 * floor[k], (k, q)
    # Find Peaks (Sec. 3.4) on the GPU's own score map, checked by the property
    # that defines the greedy result: peak k holds the largest score among the
    # valid voxels farther than 2r from peaks 0..k-1 (ties: smallest index)
    pv = res.peak_vals.cpu().numpy()
    smap = res.score.cpu().numpy()
    assert np.array_equal(pv, smap[peaks[:, 0], peaks[:, 1], peaks[:, 2]])
    lo, hi = T.valid_bounds(wl.volume.shape, L)
    m = np.full(smap.shape, -np.inf, dtype=np.float32)
    box = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
    m[box] = smap[box]
    D = 2 * r
    R = int(np.ceil(D))
    for k in range(len(peaks)):
        top = m.max()
        assert pv[k] == top, k
        first = np.flatnonzero(m.ravel() == top)[0]
        assert first == np.ravel_multi_index(tuple(peaks[k]), smap.shape), k
        z, y, x = peaks[k]
        sl = tuple(slice(max(c - R, 0), min(c + R + 1, s_)) for c, s_ in zip((z, y, x), smap.shape))
        gz, gy, gx = np.meshgrid(*[np.arange(q.start, q.stop) for q in sl], indexing="ij")
        near = (gz - z) ** 2 + (gy - y) ** 2 + (gx - x) ** 2 < D * D
        m[sl][near] = -np.inf


def test_full_size_bf16_field_c2(T, ctx):
    """BF16 storage of the tensor field (FFTs, accumulation and the variance in
    FP32/FP64, only the stored C planes rounded to bfloat16, nearest even) on
    the 256^3 workload's single 256^3 transform, in the benchmark's launch
    configuration.  The oracle rounds its own FP64 field to bfloat16 the same
    way: the score must match that within one bfloat16 step of the components
    (a component whose FP32 and FP64 values round to neighbouring bfloat16
    values moves the score by at most 2^-8 of that component; 4e-3 of the
    floor), and the FP64 score within the storage error bound 1e-2 of the floor.
    Orientations are classified against the oracle's converged multistart
    answer on the rounded field (Sec. 3.1), with lambda tolerances of one
    bfloat16 step (4e-3 of the floor)."""
    name = "c2_256cube_n6"
    say(f"[fullsize {name} bf16] generating")
    p = synth.CONFIGS[name]
    n, L, r = p["degree"], p["L"], p["mask_radius"]
    wl, Q, Tt = workload(name)
    d = T.make_desc(n, L, r)
    Tg, _ = T.build_tensor(ctx, d, cuda(wl.template), cuda(Q))
    spec = T.template_spectra(ctx, d, Tg, FFT_TILE[name])
    starts = synth.start_vectors()
    eng = T.Engine(ctx, d, spec, FFT_TILE[name], wl.volume.shape, cuda(starts),
                   field_dtype=torch.bfloat16)
    say(f"[fullsize {name} bf16] GPU pass over {len(eng.boxes)} tiles")
    res = eng.run(cuda(wl.volume), top_p=50)
    torch.cuda.synchronize()
    peaks = res.peaks.cpu().numpy().astype(np.int64)
    pts = sample_points(T, eng, wl.volume.shape, L, peaks[:16], 60, 23)
    idx = (pts[:, 0], pts[:, 1], pts[:, 2])
    sg = res.score.cpu().numpy()[idx]
    lg = res.lam.cpu().numpy()[idx]
    ug = res.direction.cpu().numpy()[idx]
    say(f"[fullsize {name} bf16] oracle on {len(pts)} voxels")
    wo, Co = oracle_field(wl.volume, pts, L, r, Tt)
    Cb = omlp.bf16_round(Co)
    so = orc.score(Co.T, n)
    sb = orc.score(Cb.T, n)
    floor = np.maximum(so, np.median(so))
    assert np.max(np.abs(sg - sb) / floor) < 4e-3
    assert np.max(np.abs(sg - so) / floor) < 1e-2
    st = starts.astype(np.float64)
    counts = {"agree": 0, "near": 0}
    for i in range(len(pts)):
        if i % 20 == 0:
            say(f"[fullsize {name} bf16] oracle orientation {i}/{len(pts)}")
        lam_o, u_o, *_ = orc.orient_multistart(Cb[i], n, st)
        cls, info = classify_orientation(Cb[i], n, lg[i], ug[i], lam_o, u_o, 40.0 * floor[i])
        assert cls is not None, (i, pts[i], info)
        counts[cls] += 1
    say(f"[fullsize {name} bf16] orientation at {len(pts)} voxels: {counts}")
    assert counts["agree"] >= 0.8 * len(pts)
