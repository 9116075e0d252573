"""Batches of uneven subtomograms with several templates in one HIP graph.

Checks: the graph replays (three, with eager work and synchronisation in
between) reproduce the eager batch bit for bit; each item equals the
stand-alone full pass of the same volume; the host-sync-free Find Peaks
equals the synchronising one on shared maps.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import require_gpu

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


@pytest.mark.parametrize("seed,shape,P,D", [(1, (20, 23, 26), 40, 3.0), (4, (33, 30, 31), 300, 4.5),
                                            # the map of the oracle-checked case of the
                                            # same shape: the all-voxel walk takes its
                                            # rounds and the final pass
                                            (5, (40, 52, 60), 2000, 6.0),
                                            (6, (6, 37, 1100), 300, 4.5)])
def test_async_peaks_equal_sync_peaks(T, ctx, seed, shape, P, D):
    rng = np.random.default_rng(seed)
    s = cuda(np.round(rng.uniform(0, 1, shape), 3).astype(np.float32))
    lo, hi = (1, 2, 3), (shape[0] - 2, shape[1] - 1, shape[2] - 4)
    pk, pv = T.find_peaks(ctx, s, lo, hi, P, D)
    peaks = torch.zeros((P, 3), dtype=torch.int32, device="cuda")
    vals = torch.zeros(P, dtype=torch.float32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    d = T.make_desc(2, 4, 1.0)
    ws = T._ws(d, 4, 32, shape, device="cuda")
    T.find_peaks_async(ctx, s, lo, hi, P, D, peaks, vals, nf, ws)
    n = int(nf.item())
    assert n == pk.shape[0]
    assert torch.equal(peaks[:n], pk) and torch.equal(vals[:n], pv)


def _batch(T, ctx, branches=4):
    rng = np.random.default_rng(11)
    templates, tmodels = [], []
    for i, (L, r) in enumerate([(12, 5.0), (16, 7.0)]):
        tm = synth.blob_template(np.random.default_rng(100 + i), L, 3)
        Q = synth.rotation_samples(5)
        d = T.make_desc(4, L, r)
        Tg, _ = T.build_tensor(ctx, d, cuda(tm.volume()), cuda(Q))
        templates.append((d, Tg))
        tmodels.append(tm)
    shapes = [(40, 40, 40), (48, 44, 52), (64, 64, 64), (36, 60, 41)]
    owner = [0, 1, 0, 1]
    vols = [rng.standard_normal(s).astype(np.float32) for s in shapes]
    for v, o in zip(vols, owner):
        tm = tmodels[o]
        c = np.array(v.shape) // 2
        rot = synth.random_rotations(rng, 1)
        v += 3.0 * synth.render_copies(v.shape, tm, c[None], rot)
    starts = cuda(synth.start_vectors())
    be = T.BatchEngine(ctx, templates, shapes, owner, starts, top_p=3, branches=branches)
    return be, vols, templates, shapes, owner, starts


def test_batch_graph_replays_match_eager_and_single_passes(T, ctx):
    be, vols, templates, shapes, owner, starts = _batch(T, ctx)
    for i, v in enumerate(vols):
        be.volumes[i].copy_(cuda(v))
    be.run_eager()
    torch.cuda.synchronize()
    ref = [(be.score[i].clone(), be.lam[i].clone(), be.direction[i].clone(), be.peaks[i].clone(),
            int(be.n_found[i].item())) for i in range(len(shapes))]
    # each item equals the stand-alone engine on the same volume
    for i, s in enumerate(shapes):
        d, Tg = templates[owner[i]]
        spec = T.template_spectra(ctx, d, Tg, be.fft[i])
        eng = T.Engine(ctx, d, spec, be.fft[i], s, starts)
        res = eng.run(cuda(vols[i]), top_p=3)
        assert torch.equal(res.score, ref[i][0])
        assert torch.equal(res.lam, ref[i][1])
        assert torch.equal(res.direction, ref[i][2])
        assert torch.equal(res.peaks, ref[i][3][:ref[i][4]])
    be.capture()
    for rep in range(3):
        for i in range(len(shapes)):
            be.score[i].zero_()
            be.lam[i].zero_()
            be.direction[i].zero_()
        be.n_found.zero_()
        _ = torch.randn(1000, device="cuda").sum().item()        # eager work between replays
        be.replay()
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(be.score[i], ref[i][0]), (rep, i)
            assert torch.equal(be.lam[i], ref[i][1]), (rep, i)
            assert torch.equal(be.direction[i], ref[i][2]), (rep, i)
            assert int(be.n_found[i].item()) == ref[i][4]
            assert torch.equal(be.peaks[i], ref[i][3]), (rep, i)


def test_batch_branch_count_does_not_change_outputs(T, ctx):
    """The items' correlation chains on 1, 3 or 4 graph branches give the
    same fields, maps and peaks bit for bit, over two replays."""
    outs = []
    for branches in (1, 3, 4):
        be, vols, *_ = _batch(T, ctx, branches=branches)
        assert be.branches == branches
        assert sorted(i for b in be.branch_items for i in b) == list(range(len(be.shapes)))
        for i, v in enumerate(vols):
            be.volumes[i].copy_(cuda(v))
        be.capture()
        for _ in range(2):
            be.replay()
        torch.cuda.synchronize()
        outs.append([torch.cat([be.Cslice[i].reshape(-1).float(), be.score[i].reshape(-1),
                                be.lam[i].reshape(-1), be.direction[i].reshape(-1),
                                be.peaks[i].reshape(-1).float()]) for i in range(len(be.shapes))])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


@pytest.mark.parametrize("learned", [False, True])
def test_quaternion_extract_batch_equals_per_box_extract(T, ctx, learned):
    """The quaternion form (d' = 4, degree 4, K = 35, four floats per
    direction) through ttm_extract_batch gives, voxel for voxel, exactly what
    ttm_extract gives for each box on its own: the multistart search, and the
    learned start with its fallback."""
    from oracle import mlp as omlp
    from oracle import sym
    from tests.gpu_common import oracle_trained_params
    n, D, K = 4, 4, 35
    d = T.make_desc(n, 12, 5.0, dprime=D)
    starts = cuda(synth.start_vectors(count=32, dim=D))
    net = (T.MLP(ctx, d, cuda(omlp.pad_params(oracle_trained_params(21, n, d=D), K, D)))
           if learned else None)
    rng = np.random.default_rng(43)
    boxes = [(5, 7, 9), (1, 1, 37), (12, 3, 20), (8, 8, 8)]
    dims = [(9, 12, 14), (3, 4, 40), (16, 5, 22), (8, 8, 8)]
    lows = [(2, 3, 4), (1, 2, 1), (0, 1, 2), (0, 0, 0)]
    entries, singles = [], []
    for box, dm, lo in zip(boxes, dims, lows):
        nv = int(np.prod(box))
        q = rng.standard_normal((nv, D))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        Cb = cuda((sym.monomials(q, n) + 0.25 * rng.standard_normal((nv, K))).T.reshape(K, *box))
        maps = [torch.zeros(dm, device="cuda"), torch.zeros(dm, device="cuda"),
                torch.zeros((*dm, D), device="cuda")]
        entries.append(dict(C=Cb, score=maps[0], lam=maps[1], direction=maps[2], out_lo=lo))
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        s1, l1, u1 = T.extract(ctx, d, Cb, starts=starts, out_lo=lo, out_dims=dm, mlp=net, kappa=0.3,
                               fallbacks=fb)
        assert u1.shape[-1] == D
        singles.append((s1, l1, u1, int(fb.item())))
    eb = T.ExtractBatch(ctx, d, entries)
    ws = torch.empty(eb.workspace_bytes(), dtype=torch.uint8, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    eb.run(starts, ws, mlp=net, kappa=0.3, fallbacks=fb)
    torch.cuda.synchronize()
    for e, (s1, l1, u1, f1) in zip(entries, singles):
        assert torch.equal(e["score"], s1) and torch.equal(e["lam"], l1) and torch.equal(e["direction"], u1)
    assert int(fb.item()) == sum(x[3] for x in singles)
    if learned:
        assert int(fb.item()) < sum(int(np.prod(b)) for b in boxes)


def test_pick_fft_and_tiles(T):
    assert T.tiles_for((96, 96, 96), 40, 128) == 1
    assert T.tiles_for((192, 192, 192), 40, 128) == 8
    assert T.tiles_for((192, 192, 192), 40, 192) == 1
    # default model N^3 log2 N: one 96^3 tile beats one 128^3 tile
    assert T.pick_fft((96, 96, 96), 40) == 96
    # one 192^3 tile (5.4e7) beats eight 128^3 tiles (1.2e8) and four 160^3 tiles (1.2e8)
    assert T.pick_fft((192, 160, 192), 24) == 192
    # with measured costs only the measured edges compete; cheap small tiles win
    assert T.pick_fft((192, 192, 192), 40, {64: 0.001, 128: 1.0, 256: 100.0, 512: 1e4}) == 64
    assert T.pick_fft((192, 192, 192), 40, {128: 1.0, 192: 2.0}) == 192


def test_batch_c5_shapes_match_oracle(T, ctx):
    """Subtomograms of the 64-item batch's recipe (edges 96..192, degree 6,
    three templates of edges 24, 32, 40), run as one graph: at sampled voxels
    of every item (its peaks and random valid voxels) w, the score and the
    orientation against the FP64 oracle's direct sums (Eq. norm_f, Eq. tcc,
    Sec. 3.1, 3.2), with the tolerances of the single-volume tests."""
    from oracle import sym, ttm as orc
    from tests.gpu_common import classify_orientation
    print("[batch c5 shapes] generating", flush=True)
    tmpls, items = synth.batch_items(seed=5, n_items=64)
    # the first item of each edge
    pick = [next(k for k, it in enumerate(items) if it["volume"].shape[0] == e)
            for e in (96, 128, 160, 192)]
    n = 6
    Q = synth.rotation_samples(10)
    templates, oracle_T = [], []
    for vol_t, r, tm in tmpls:
        d = T.make_desc(n, vol_t.shape[0], r)
        Tg, _ = T.build_tensor(ctx, d, cuda(vol_t), cuda(Q))
        templates.append((d, Tg))
        oracle_T.append(orc.tensor_template(orc.normalize_template(vol_t.astype(np.float64), r), Q, n))
    shapes = [items[k]["volume"].shape for k in pick]
    owner = [items[k]["template"] for k in pick]
    starts = synth.start_vectors()
    be = T.BatchEngine(ctx, templates, shapes, owner, cuda(starts), top_p=8)
    for i, k in enumerate(pick):
        be.volumes[i].copy_(cuda(items[k]["volume"]))
    be.capture()
    be.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    counts = {"agree": 0, "near": 0}
    for i, k in enumerate(pick):
        vol = items[k]["volume"]
        d = templates[owner[i]][0]
        L, r = d.L, d.mask_radius
        print(f"[batch c5 shapes] item {i}: {shapes[i]}, L={L}, FFT edge {be.fft[i]}", flush=True)
        lo, hi = T.valid_bounds(shapes[i], L)
        nf = int(be.n_found[i].item())
        pts = np.concatenate([be.peaks[i][:nf].cpu().numpy().astype(np.int64),
                              np.stack([rng.integers(a, b + 1, 10) for a, b in zip(lo, hi)], 1)])
        c = L // 2
        patches = np.stack([orc.prefilter_box(vol, (z - c, y - c, x - c), (z - c + L, y - c + L, x - c + L))
                            for z, y, x in pts])
        g2 = orc.volume_g2_mean(orc.prefilter_volume(vol))
        wo, Co = orc.field_at(patches, orc.ball_mask(L, r), oracle_T[owner[i]], g2)
        idx = (pts[:, 0], pts[:, 1], pts[:, 2])
        sg = be.score[i].cpu().numpy()[idx]
        lg = be.lam[i].cpu().numpy()[idx]
        ug = be.direction[i].cpu().numpy()[idx]
        so = orc.score(Co.T, n)
        floor = np.maximum(so, np.median(so))
        assert np.all(wo > 0)
        assert np.max(np.abs(sg - so) / floor) < 1e-4, i
        for j in range(len(pts)):
            lam_o, u_o, *_ = orc.orient_multistart(Co[j], n, starts.astype(np.float64))
            cls, info = classify_orientation(Co[j], n, lg[j], ug[j], lam_o, u_o, floor[j])
            assert cls is not None, (i, pts[j], info)
            counts[cls] += 1
        # the peaks are the greedy result on the item's own map (Sec. 3.4)
        smap = be.score[i].cpu().numpy().astype(np.float64)
        full = np.zeros_like(smap)
        box = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
        full[box] = smap[box]
        pko, _ = orc.find_peaks(full, lo, hi, 8, 2 * r)
        assert np.array_equal(be.peaks[i][:nf].cpu().numpy().astype(np.int64), pko)
    print(f"[batch c5 shapes] orientation {counts}", flush=True)
    total = sum(counts.values())
    assert counts["agree"] >= 0.8 * total


def test_peak_batch_equals_find_peaks_per_map(T, ctx):
    """Find Peaks over several maps in one launch (ttm_find_peaks_batch) gives,
    for each map, exactly the peaks and values of ttm_find_peaks (Sec. 3.4),
    on maps with many exact ties, including a map where P is out of reach."""
    cases = [(1, (20, 23, 26), 40, 3.0), (2, (40, 41, 42), 200, 5.5), (3, (9, 10, 11), 300, 1.0),
             (5, (40, 52, 60), 2000, 6.0), (6, (64, 70, 50), 60, 20.0), (7, (20, 18, 19), 7, 0.0)]
    entries, maps = [], []
    for seed, shape, P, D in cases:
        rng = np.random.default_rng(seed)
        s = cuda(np.round(rng.uniform(0, 1, shape), 3).astype(np.float32))
        lo, hi = (1, 2, 3), (shape[0] - 2, shape[1] - 1, shape[2] - 4)
        maps.append((s, lo, hi, P, D))
        entries.append(dict(score=s, lo=lo, hi=hi, top_p=P, min_dist=D,
                            peaks=torch.zeros((P, 3), dtype=torch.int32, device="cuda"),
                            vals=torch.zeros(P, dtype=torch.float32, device="cuda"),
                            n_found=torch.zeros(1, dtype=torch.int32, device="cuda")))
    pb = T.PeakBatch(ctx, entries)
    for rep in range(2):                      # a second run on the same scratch
        pb.run()
        torch.cuda.synchronize()
        for (s, lo, hi, P, D), e in zip(maps, entries):
            pk, pv = T.find_peaks(ctx, s, lo, hi, P, D)
            n = int(e["n_found"].item())
            assert n == pk.shape[0], (rep, s.shape, P, D)
            assert torch.equal(e["peaks"][:n], pk) and torch.equal(e["vals"][:n], pv)


@pytest.mark.parametrize("learned", [False, True])
def test_extract_batch_equals_per_box_extract(T, ctx, learned):
    """ttm_extract_batch over boxes of different shapes (each written into its
    own maps at an offset) gives, voxel for voxel, exactly what ttm_extract
    gives for each box on its own: plain multistart and learned start with its
    fallback."""
    from oracle import mlp as omlp
    from oracle import sym
    from tests.gpu_common import oracle_trained_params
    n, K = 6, 28
    d = T.make_desc(n, 16, 7.0)
    starts = cuda(synth.start_vectors())
    net = T.MLP(ctx, d, cuda(omlp.pad_params(oracle_trained_params(12, n), K))) if learned else None
    rng = np.random.default_rng(41)
    boxes = [(5, 7, 9), (1, 1, 37), (12, 3, 20), (8, 8, 8)]
    dims = [(9, 12, 14), (3, 4, 40), (16, 5, 22), (8, 8, 8)]
    lows = [(2, 3, 4), (1, 2, 1), (0, 1, 2), (0, 0, 0)]
    entries, singles = [], []
    for box, dm, lo in zip(boxes, dims, lows):
        nv = int(np.prod(box))
        v = rng.standard_normal((nv, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        Cb = cuda((sym.monomials(v, n) + 0.3 * rng.standard_normal((nv, K))).T.reshape(K, *box))
        maps = [torch.zeros(dm, device="cuda"), torch.zeros(dm, device="cuda"),
                torch.zeros((*dm, 3), device="cuda")]
        entries.append(dict(C=Cb, score=maps[0], lam=maps[1], direction=maps[2], out_lo=lo))
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        s1, l1, u1 = T.extract(ctx, d, Cb, starts=starts, out_lo=lo, out_dims=dm, mlp=net, kappa=0.3,
                               fallbacks=fb)
        singles.append((s1, l1, u1, int(fb.item())))
    eb = T.ExtractBatch(ctx, d, entries)
    ws = torch.empty(eb.workspace_bytes(), dtype=torch.uint8, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    eb.run(starts, ws, mlp=net, kappa=0.3, fallbacks=fb)
    torch.cuda.synchronize()
    for e, (s1, l1, u1, f1) in zip(entries, singles):
        assert torch.equal(e["score"], s1) and torch.equal(e["lam"], l1) and torch.equal(e["direction"], u1)
    assert int(fb.item()) == sum(x[3] for x in singles)
