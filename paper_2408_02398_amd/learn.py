"""Learned start for the orientation search: training data, training, calibration.

The network is trained on (tensor, direction) pairs that TTM itself produces:
the tensor field C(x) of synthetic tomograms holding copies of the template,
labelled with the plain multistart answer at each sampled voxel.  Every step
runs through libttm (correlation, extraction, the BF16 training kernels);
this module only selects voxels and batches.

Calibration picks the fallback threshold kappa on held-out voxels of the
highest scores (the voxels whose orientation is used): the smallest kappa
such that among them, those whose learned lambda / ||C||_F is at least kappa
end more than 1 degree from the multistart answer at most `max_wrong` of the
time.  Voxels below kappa, not converged, or beaten by a fixed start take the
multistart fallback.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import ttm


@dataclass
class TrainingSet:
    C: torch.Tensor        # B x K raw tensors
    u: torch.Tensor        # B x d' multistart directions
    score: torch.Tensor    # B Frobenius scores


def collect(ctx, desc, spectra, fft_n, vol: torch.Tensor, starts: torch.Tensor, n_uniform: int,
            n_top: int, seed: int = 0, max_tiles: int | None = None) -> TrainingSet:
    """Sample voxels of each tile (uniform + highest score) and label them."""
    g, w, stats = ttm.normalize(ctx, desc, vol, spectra, fft_n)
    K = ttm.n_components(desc.degree, desc.dprime)
    gen = torch.Generator(device=vol.device)
    gen.manual_seed(seed)
    boxes = ttm.tile_boxes(tuple(vol.shape), desc.L, fft_n)
    if max_tiles is not None:
        boxes = boxes[:max_tiles]
    Cs, us, ss = [], [], []
    for lo, size in boxes:
        C = ttm.correlate(ctx, desc, g, w, stats, spectra, fft_n, lo, size)
        s, _, _ = ttm.extract(ctx, desc, C, orient=False)
        flat, sflat = C.view(K, -1), s.view(-1)
        nvox = sflat.numel()
        iu = torch.randint(0, nvox, (min(n_uniform, nvox),), generator=gen, device=vol.device)
        it = torch.topk(sflat, min(n_top, nvox)).indices
        idx = torch.unique(torch.cat([iu, it]))
        sample = flat[:, idx].contiguous()
        m = sample.shape[1]
        _, _, u = ttm.extract(ctx, desc, sample.view(K, 1, 1, m), starts=starts)
        Cs.append(sample.t().contiguous())
        us.append(u.view(m, desc.dprime).clone())
        ss.append(sflat[idx].clone())
    return TrainingSet(torch.cat(Cs), torch.cat(us), torch.cat(ss))


def train(net: "ttm.MLP", data: TrainingSet, steps: int = 3000, batch: int = 4096,
          lr: float = 3e-3, lr_min: float = 1e-4, seed: int = 0, log_every: int = 0) -> list:
    """Adam with cosine decay on random mini-batches; returns the loss curve."""
    gen = torch.Generator(device=data.C.device)
    gen.manual_seed(seed)
    B = data.C.shape[0]
    curve = []
    for s in range(steps):
        idx = torch.randint(0, B, (batch,), generator=gen, device=data.C.device)
        rate = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * s / max(steps - 1, 1)))
        loss = net.train_step(data.C[idx].contiguous(), data.u[idx].contiguous(), lr=float(rate))
        if log_every and (s % log_every == 0 or s == steps - 1):
            curve.append((s, float(loss.item())))
    return curve


def angles_deg(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    c = torch.abs(torch.sum(a * b, dim=-1)) / (a.norm(dim=-1) * b.norm(dim=-1)).clamp_min(1e-30)
    return torch.rad2deg(torch.arccos(c.clamp(max=1.0)))


def evaluate(ctx, desc, net, data: TrainingSet, starts, kappa: float):
    """Learned orientation on labelled voxels: (angles vs multistart, lambda / ||C||, fallbacks)."""
    K = data.C.shape[1]
    B = data.C.shape[0]
    Cb = data.C.t().contiguous().view(K, 1, 1, B)
    fb = torch.zeros(1, dtype=torch.int32, device=data.C.device)
    s, lam, u = ttm.extract(ctx, desc, Cb, starts=starts, mlp=net, kappa=kappa, fallbacks=fb)
    ang = angles_deg(u.view(B, desc.dprime), data.u)
    if desc.dprime == 4:
        ang = 2.0 * ang                          # rotation distance 2 arccos|q1.q2|
    return ang, (lam.view(B) / s.view(B).clamp_min(1e-30)), int(fb.item())


def calibrate(ctx, desc, net, data: TrainingSet, starts, max_wrong: float = 0.02) -> dict:
    """Smallest kappa whose accepted voxels are wrong (> 1 degree) at most max_wrong of the time."""
    ang, lam_hat, fb_conv = evaluate(ctx, desc, net, data, starts, kappa=-1e30)
    order = torch.argsort(lam_hat, descending=True)
    wrong = (ang[order] > 1.0).float()
    frac = torch.cumsum(wrong, 0) / torch.arange(1, len(wrong) + 1, device=wrong.device)
    ok = torch.nonzero(frac <= max_wrong).flatten()
    n_acc = int(ok.max().item()) + 1 if ok.numel() else 0
    if n_acc == len(wrong):
        kappa = float("-inf")        # every calibration voxel accepted: no lower bound is justified
    else:
        kappa = float(lam_hat[order[n_acc - 1]].item()) if n_acc > 0 else float("inf")
    return {"kappa": kappa, "accepted_fraction": n_acc / len(wrong),
            "wrong_without_fallback": float((ang > 1.0).float().mean().item()),
            "median_angle_without_fallback": float(ang.median().item()),
            "not_converged_fraction": fb_conv / len(wrong)}


def init_params(K: int, seed: int = 0, device="cuda", dout: int = 3) -> torch.Tensor:
    """He-normal initial master parameters in the kernels' layout (W1 [kin][64],
    kin = 32 for K <= 32 else 48; dout = d' outputs; random inputs, host-drawn)."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((32 if K <= 32 else 48, 64))
    W1[:K] = rng.standard_normal((K, 64)) * np.sqrt(2.0 / K)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    W3 = np.zeros((64, 16))
    W3[:, :dout] = rng.standard_normal((64, dout)) * np.sqrt(1.0 / 64)
    flat = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.zeros(16)])
    return torch.from_numpy(flat.astype(np.float32)).to(device)


def build_learned_start(ctx, desc, spectra, fft_n, tomograms, starts, *, n_uniform=60000,
                        n_top=60000, steps=6000, batch=8192, lr=3e-3, max_wrong=0.03, seed=0,
                        log=print) -> tuple:
    """Collect on all but the last tomogram, train, calibrate kappa on the last one."""
    t0 = time.time()
    train_sets = [collect(ctx, desc, spectra, fft_n, v, starts, n_uniform, n_top, seed + i)
                  for i, v in enumerate(tomograms[:-1])]
    data = TrainingSet(torch.cat([d.C for d in train_sets]), torch.cat([d.u for d in train_sets]),
                       torch.cat([d.score for d in train_sets]))
    held = collect(ctx, desc, spectra, fft_n, tomograms[-1], starts, 0, n_top, seed + 99)
    held_u = collect(ctx, desc, spectra, fft_n, tomograms[-1], starts, n_uniform, 0, seed + 98)
    torch.cuda.synchronize()
    t1 = time.time()
    K = ttm.n_components(desc.degree, desc.dprime)
    net = ttm.MLP(ctx, desc, init_params(K, seed, device=spectra.device, dout=desc.dprime))
    curve = train(net, data, steps=steps, batch=batch, lr=lr, seed=seed, log_every=max(steps // 10, 1))
    torch.cuda.synchronize()
    t2 = time.time()
    cal = calibrate(ctx, desc, net, held, starts, max_wrong=max_wrong)
    ang_u, _, fb_u = evaluate(ctx, desc, net, held_u, starts, kappa=cal["kappa"])
    ang_t, _, fb_t = evaluate(ctx, desc, net, held, starts, kappa=cal["kappa"])
    cal.update({"heldout_top_within_1deg": float((ang_t <= 1.0).float().mean().item()),
                "heldout_top_fallback": fb_t / len(ang_t),
                "heldout_uniform_within_1deg": float((ang_u <= 1.0).float().mean().item()),
                "heldout_uniform_fallback": fb_u / len(ang_u)})
    info = {"train_samples": int(data.C.shape[0]), "heldout_samples": int(held.C.shape[0]),
            "collect_s": t1 - t0, "train_s": t2 - t1, "loss_curve": curve, **cal}
    log(f"[learn] {info}")
    return net, cal["kappa"], info
