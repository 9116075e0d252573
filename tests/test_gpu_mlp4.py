"""GPU parity of the learned start of the quaternion form (d' = 4, degree 4:
K = 35 features, so the 48-input network, with 4 outputs) against the FP64
oracle: training on the matrix cores, the learned orientation path (SS-HOPM
from the network's quaternion, the Newton polish, the certification, the
screen and the multistart fallback) against the oracle's reading of it, and
the exact merge of the fallback.  Orientations are classified as in
test_gpu_parity (within 1 degree, or a near-optimal maximiser of the FP64
function, or, where a fallback test is within rounding of flipping, the
other branch's answer).
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import sym, ttm as orc
from tests.gpu_common import classify_orientation, oracle_trained_params, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, D = 4, 4
K = 35


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


def rank_one_quaternions(rng, B, noise=0.15):
    q = rng.standard_normal((B, D))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q, sym.monomials(q, N) + noise * rng.standard_normal((B, K))


def test_quaternion_network_layout_and_training(T, ctx):
    """The 48-input network: the master layout holds W1 [48][64]; training on
    rank-one quaternion tensors (target q) lowers the sign-invariant loss, and
    the padded rows and columns stay zero."""
    print("[mlp d'=4] training", flush=True)
    d = T.make_desc(N, 12, 5.0, dprime=4)
    p = omlp.init_params(np.random.default_rng(3), K, d_out=D)
    flat = omlp.pad_params(p, K, D)
    assert flat.size == 48 * 64 + 64 + 64 * 64 + 64 + 64 * 16 + 16
    net = T.MLP(ctx, d, cuda(flat))
    assert net.n_params == flat.size
    rng = np.random.default_rng(4)
    q, C = rank_one_quaternions(rng, 4096)
    Cg, tg = cuda(C), cuda(q)
    first = float(net.train_step(Cg, tg, lr=3e-3).item())
    for _ in range(300):
        last = net.train_step(Cg, tg, lr=3e-3)
    last = float(last.item())
    print(f"[mlp d'=4] loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.3 * first
    got = omlp.unpad_params(net.params.cpu().numpy(), K, D)
    full = net.params.cpu().numpy()
    assert np.all(full[K * 64:48 * 64] == 0.0)                      # W1 rows >= K
    w3 = full[48 * 64 + 64 + 64 * 64 + 64:][:64 * 16].reshape(64, 16)
    assert np.all(w3[:, D:] == 0.0) and np.all(got["b3"] == got["b3"])


def test_quaternion_learned_path_matches_oracle(T, ctx):
    print("[mlp d'=4] learned path", flush=True)
    d = T.make_desc(N, 12, 5.0, dprime=4)
    pl = oracle_trained_params(21, N, d=D)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(pl, K, D)))
    rng = np.random.default_rng(22)
    Bt = 96
    _, Ct = rank_one_quaternions(rng, Bt, noise=0.25)
    starts = synth.start_vectors(count=32, dim=4)
    kappa = 0.3
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _, lam, u = T.extract(ctx, d, cuda(Ct.T.reshape(K, 1, 1, Bt)), starts=cuda(starts), mlp=net,
                          kappa=kappa, fallbacks=fb)
    lg, ug = lam.cpu().numpy().ravel(), u.cpu().numpy().reshape(Bt, D)
    st64 = starts.astype(np.float64)
    counts = {"agree": 0, "near": 0, "alt": 0}
    nfb = 0
    for i in range(Bt):
        lo, uo, fell, info = omlp.orient_learned(Ct[i], N, pl, st64, kappa, detail=True,
                                                 newton_first=0)
        nfb += fell
        cn = orc.score(Ct[i], N, D)
        alts = []
        if (abs(info["beat_gap"]) < 1e-4 * cn or abs(info["kappa_gap"]) < 1e-4
                or abs(info["cert_step"] - 1e-2) < 3e-3):
            alts.append((info["lam_learned"], info["u_learned"]))
            alts.append(orc.orient_multistart(Ct[i], N, st64)[:2])
        cls, det = classify_orientation(Ct[i], N, lg[i], ug[i], lo, uo, cn, alts)
        assert cls is not None, (i, det, info["beat_gap"], info["kappa_gap"], info["cert_step"])
        assert ug[i][0] >= 0
        counts[cls] += 1
    print(f"[mlp d'=4 learned path {Bt} voxels] {counts}, fallbacks oracle {nfb} gpu {int(fb.item())}",
          flush=True)
    assert counts["agree"] >= 0.8 * Bt
    assert abs(int(fb.item()) - nfb) <= 2


def test_quaternion_forced_fallback_equals_multistart(T, ctx):
    """kappa = +inf sends every voxel to the multistart fallback; the merged
    answer is, bit for bit, the larger of the learned-only answer (kappa =
    -inf, no screening) and the plain multistart answer."""
    print("[mlp d'=4] forced fallback", flush=True)
    B = 160
    rng = np.random.default_rng(23)
    C = rng.standard_normal((B, K))
    d = T.make_desc(N, 12, 5.0, dprime=4)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(oracle_trained_params(24, N, steps=50, d=D), K, D)))
    starts = cuda(synth.start_vectors(count=32, dim=4))
    Cg = cuda(C.T.reshape(K, 1, 1, B))
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _, lam_m, u_m = T.extract(ctx, d, Cg, starts=starts, mlp=net, kappa=float("inf"), fallbacks=fb)
    assert int(fb.item()) == B
    _, lam_l, u_l = T.extract(ctx, d, Cg, starts=starts, mlp=net, kappa=float("-inf"), screen=False)
    _, lam_p, u_p = T.extract(ctx, d, Cg, starts=starts)
    lm, ll, lp = (x.cpu().numpy().ravel() for x in (lam_m, lam_l, lam_p))
    um, ul, up = (x.cpu().numpy().reshape(B, D) for x in (u_m, u_l, u_p))
    plain_wins = lp > ll
    assert np.array_equal(lm, np.where(plain_wins, lp, ll))
    assert np.array_equal(um, np.where(plain_wins[:, None], up, ul))
    print(f"[mlp d'=4 forced fallback] plain larger at {int(plain_wins.sum())} of {B}", flush=True)
