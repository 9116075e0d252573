"""What the trained network gains over the method without it (the learned
start's extension of Sec. 3.1's seeds), on a held-out synthetic tomogram.

The network is trained by the library's own BF16 kernels on (tensor,
multistart direction) pairs that TTM generates from three training tomograms
of the template, its fallback threshold calibrated on a fourth; the held-out
tomogram (another seed) is then scored three ways, each a full pass through
the C ABI: plain 16-start multistart, the learned start with the trained
network, and the learned start with the untrained (initial) network.  The
trained network must (1) send fewer voxels to the multistart fallback than the
untrained one, (2) keep the median angle to the plain answer at <= 1 degree
on the voxels that matter (top 1% scores and r_s = 3 spheres around the
peaks, Sec. 3.3), with the same peaks, and (3) make the pass faster than the
plain multistart.
"""
import numpy as np
import pytest

import synth
from tests.gpu_common import require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


def test_trained_network_gains_over_untrained_and_plain():
    require_gpu()
    from paper_2408_02398_amd import learn, ttm
    ctx = ttm.Context(0)
    n, L, r, N = 6, 32, 14.0, 128
    shape = (128, 128, 128)

    def tomo(seed):
        return synth.make_tomogram(f"gain{seed}", shape, L=L, n_blobs=4, n_copies=12, min_sep=L,
                                   mask_radius=r, degree=n, seed=seed, snr=0.1, wedge=True,
                                   template_seed=2)
    say("[gain] generating tomograms")
    train = [tomo(300 + i) for i in range(4)]
    held = tomo(399)
    assert all(np.array_equal(t.template, held.template) for t in train)
    d = ttm.make_desc(n, L, r)
    Q = torch.from_numpy(synth.rotation_samples(40)).float().cuda()
    Tg, _ = ttm.build_tensor(ctx, d, torch.from_numpy(held.template).cuda(), Q)
    spec = ttm.template_spectra(ctx, d, Tg, N)
    starts = torch.from_numpy(synth.start_vectors()).cuda()
    vols = [torch.from_numpy(t.volume).cuda() for t in train]
    say("[gain] training")
    net, kappa, info = learn.build_learned_start(ctx, d, spec, N, vols, starts, n_uniform=20000,
                                                 n_top=20000, steps=4000, batch=4096, log=say)
    K = ttm.n_components(n, 3)
    untrained = ttm.MLP(ctx, d, learn.init_params(K, 0))
    vol = torch.from_numpy(held.volume).cuda()

    def run(mlp, kap):
        eng = ttm.Engine(ctx, d, spec, N, shape, starts, mlp=mlp, kappa=kap)
        eng.run(vol, top_p=12)                       # warm-up
        torch.cuda.synchronize()
        eng.fallbacks.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        res = eng.run(vol, top_p=12)
        b.record()
        torch.cuda.synchronize()
        return res, a.elapsed_time(b), int(eng.fallbacks.item())

    say("[gain] held-out passes")
    plain, t_plain, _ = run(None, 0.0)
    plain = (plain.score.clone(), plain.direction.clone(), plain.peaks.clone())
    tr, t_tr, fb_tr = run(net, kappa)
    tr = (tr.direction.clone(), tr.peaks.clone())
    un, t_un, fb_un = run(untrained, kappa)
    say(f"[gain] ms plain {t_plain:.2f} trained {t_tr:.2f} untrained {t_un:.2f}; "
        f"fallbacks trained {fb_tr} untrained {fb_un}; kappa {kappa}")
    # the voxels that matter: top 1% of valid scores and r_s = 3 spheres around the peaks
    lo, hi = ttm.valid_bounds(shape, L)
    sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
    sv = plain[0][sl]
    thr = torch.quantile(sv.reshape(-1)[::7], 0.99)
    mask = torch.zeros_like(plain[0], dtype=torch.bool)
    mask[sl] = sv >= thr
    rs = 3
    g = torch.arange(-rs, rs + 1, device="cuda")
    offs = torch.stack(torch.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    offs = offs[(offs ** 2).sum(1) <= rs * rs]
    pts = (plain[2].long()[:, None, :] + offs[None]).reshape(-1, 3)
    for a_ in range(3):
        pts[:, a_] = pts[:, a_].clamp(lo[a_], hi[a_])
    mask[pts[:, 0], pts[:, 1], pts[:, 2]] = True
    ua, ub = plain[1][mask], tr[0][mask]
    c = torch.abs((ua * ub).sum(-1)).clamp(max=1.0)
    med = float(torch.rad2deg(torch.arccos(c)).median().item())
    say(f"[gain] median angle trained vs plain on {int(mask.sum())} voxels: {med:.4f} deg")
    assert fb_tr < fb_un
    assert med <= 1.0
    assert torch.equal(tr[1], plain[2])
    assert t_tr < t_plain
