"""The paper's robustness experiment in small (Sec. 4.1, rotation deviation
against SNR): a 3 x 3 x 3 grid of randomly rotated copies of a 32^3 blob
template at SNR 10 and 0.3, quaternion form at degree 4.  A full pass, Find
Peaks and TTM-ref (Alg. 3); each planted copy is matched to its nearest peak.

Checks against the planted truth (no oracle involved; these pin the method's
behaviour end to end): every copy is found; TTM-ref puts every copy on its
exact centre; its mean rotation error 2 arccos|q1.q2| is under 1.5 degrees at
SNR 10 and grows as the noise grows (the paper: under 1 degree for SNR > 1,
worse at low SNR)."""
import numpy as np
import pytest

import synth
from tests.gpu_common import require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
torch = pytest.importorskip("torch")


def test_noise_sweep_small():
    require_gpu()
    from paper_2408_02398_amd import ttm
    ctx = ttm.Context(0)
    n, L, r, N = 4, 32, 14.0, 128
    d = ttm.make_desc(n, L, r, dprime=4)
    Q = torch.from_numpy(synth.rotation_samples(400)).float().cuda()
    starts = torch.from_numpy(synth.start_vectors(count=32, dim=4)).cuda()
    means = []
    for k, snr in enumerate((10.0, 0.3)):
        wl = synth.grid_tomogram(f"sw{snr:g}", 3, 40, L, 4, r, n, seed=700 + k, snr=snr,
                                 template_seed=2)
        if k == 0:
            T, tn = ttm.build_tensor(ctx, d, torch.from_numpy(wl.template).cuda(), Q)
            spec = ttm.template_spectra(ctx, d, T, N)
        eng = ttm.Engine(ctx, d, spec, N, wl.volume.shape, None, orient=False)
        res = eng.run(torch.from_numpy(wl.volume).cuda(), top_p=27)
        ref = ttm.refine(ctx, d, res.g, res.w, T, tn, res.peaks.contiguous(), starts, r_s=3.0)
        pk = res.peaks.cpu().numpy().astype(np.float64)
        pos = ref["pos"].cpu().numpy().astype(np.float64)
        quat = ref["quat"].cpu().numpy()
        errs = []
        for c, qt in zip(wl.centres.astype(np.float64), wl.quaternions):
            dist = np.linalg.norm(pk - c, axis=1)
            i = int(np.argmin(dist))
            assert dist[i] <= r
            assert np.array_equal(pos[i], c), (snr, c, pos[i])
            cq = abs(float(np.dot(quat[i] / np.linalg.norm(quat[i]), qt)))
            errs.append(np.degrees(2 * np.arccos(min(1.0, cq))))
        means.append(float(np.mean(errs)))
        print(f"[sweep] SNR {snr}: TTM-ref rotation error mean {means[-1]:.2f} max {max(errs):.2f} deg",
              flush=True)
    assert means[0] < 1.5
    assert means[1] > means[0]
