"""GPU parity of the learned start: BF16 matrix-core inference and training
kernels against the FP64 network of the oracle, and the learned orientation
path (with its multistart fallback) against the oracle's reading of it.

Tolerances: start directions within 0.05 degrees of the oracle's forward pass
with BF16 rounding emulated; gradients normwise within 1e-2 of the FP64
backward (the kernels also round gradients to BF16 as matrix-core operands);
orientations as in test_gpu_parity.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import sym, ttm as orc
from tests.gpu_common import classify_orientation, oracle_trained_params, require_gpu

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


def oracle_params(seed, K=28, bias=0.1):
    rng = np.random.default_rng(seed)
    p = omlp.init_params(rng, K)
    for k in ("b1", "b2", "b3"):
        p[k] = bias * rng.standard_normal(p[k].shape)
    return p


def test_param_layout_roundtrip():
    p = oracle_params(0)
    q = omlp.unpad_params(omlp.pad_params(p, 28), 28)
    for k in p:
        assert np.array_equal(p[k], q[k])


@pytest.mark.parametrize("n", [4, 6])
def test_learned_start_inference_matches_oracle(T, ctx, n):
    K = sym.n_components(n, 3)
    p = oracle_params(1, K)
    d = T.make_desc(n, 16, 7.0)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(p, K)))
    B = 300
    rng = np.random.default_rng(2)
    C = rng.standard_normal((B, K))
    C[7] = 0.0                                    # zero tensor: start = first fixed start
    Cg = cuda(C.T.reshape(K, 1, 1, B))
    _, _, u = T.extract(ctx, d, Cg, starts=cuda(synth.start_vectors()), mlp=net, start_only=True)
    ug = u.cpu().numpy().reshape(B, 3).astype(np.float64)
    y, _ = omlp.forward(p, omlp.features(C, n), bf16=True)
    uo = y / np.linalg.norm(y, axis=1, keepdims=True)
    ok = np.ones(B, bool)
    ok[7] = False
    cosv = np.sum(ug[ok] * uo[ok], axis=1)
    assert np.degrees(np.arccos(np.clip(np.min(cosv), -1, 1))) < 0.05


def test_training_gradients_match_oracle(T, ctx):
    n, K, B = 6, 28, 512
    p = oracle_params(3, K)
    d = T.make_desc(n, 16, 7.0)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(p, K)))
    rng = np.random.default_rng(4)
    C = rng.standard_normal((B, K))
    t = rng.standard_normal((B, 3))
    grads = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    loss = net.train_step(cuda(C), cuda(t), lr=0.0, grads=grads)
    pr = {k: (omlp.bf16_round(v) if k.startswith("W") else v) for k, v in p.items()}
    y, cache = omlp.forward(pr, omlp.features(C, n), bf16=True)
    go = omlp.backward(pr, cache, t)
    gg = omlp.unpad_params(grads.cpu().numpy(), K)
    assert float(loss.item()) == pytest.approx(omlp.loss(y, t), rel=1e-3)
    for k in go:
        err = np.linalg.norm(gg[k] - go[k]) / np.linalg.norm(go[k])
        assert err < 1e-2, (k, err)
    # padding stays zero
    flat = grads.cpu().numpy()
    assert np.all(flat[K * 64:32 * 64] == 0)


def test_adam_step_matches_oracle(T, ctx):
    n, K, B = 6, 28, 256
    p = oracle_params(5, K)
    d = T.make_desc(n, 16, 7.0)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(p, K)))
    rng = np.random.default_rng(6)
    C, t = rng.standard_normal((B, K)), rng.standard_normal((B, 3))
    grads = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    net.train_step(cuda(C), cuda(t), lr=1e-2, grads=grads)
    # first Adam step: p - lr * g / (|g| + eps) elementwise, with the kernel's own gradient
    g = grads.cpu().numpy().astype(np.float64)
    p0 = omlp.pad_params(p, K)
    want = p0 - 1e-2 * g / (np.abs(g) + 1e-8)
    got = net.params.cpu().numpy().astype(np.float64)
    assert np.allclose(got, want, atol=2e-6)


def test_training_learns_and_learned_path_matches_oracle(T, ctx):
    n, K = 6, 28
    rng = np.random.default_rng(7)
    B = 4096
    v = rng.standard_normal((B, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    C = sym.monomials(v, n) + 0.15 * rng.standard_normal((B, K))
    d = T.make_desc(n, 16, 7.0)
    p = omlp.init_params(np.random.default_rng(8), K)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(p, K)))
    Cg, tg = cuda(C), cuda(v)
    first = float(net.train_step(Cg, tg, lr=3e-3).item())
    for _ in range(400):
        last = net.train_step(Cg, tg, lr=3e-3)
    last = float(last.item())
    assert last < 0.25 * first
    # learned orientation path vs the oracle's reading of it on held-out tensors;
    # both sides take the network that the oracle trained on the CPU
    pl = oracle_trained_params(12, n)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(pl, K)))
    Bt = 128
    vt = rng.standard_normal((Bt, 3))
    vt /= np.linalg.norm(vt, axis=1, keepdims=True)
    Ct = sym.monomials(vt, n) + 0.15 * rng.standard_normal((Bt, K))
    starts = synth.start_vectors()
    kappa = 0.3
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _, lam, u = T.extract(ctx, d, cuda(Ct.T.reshape(K, 1, 1, Bt)), starts=cuda(starts), mlp=net,
                          kappa=kappa, fallbacks=fb)
    lg, ug = lam.cpu().numpy().ravel(), u.cpu().numpy().reshape(Bt, 3)
    nfb = 0
    counts = {"agree": 0, "near": 0, "alt": 0}
    st64 = starts.astype(np.float64)
    for i in range(Bt):
        lo, uo, fell, info = omlp.orient_learned(Ct[i], n, pl, st64, kappa, detail=True)
        nfb += fell
        cn = orc.score(Ct[i], n)
        # a fallback test within rounding of flipping may go either way on the
        # GPU: then either branch's answer is one the method gives
        alts = []
        if (abs(info["beat_gap"]) < 1e-4 * cn or abs(info["kappa_gap"]) < 1e-4
                or abs(info["cert_step"] - 1e-2) < 3e-3):
            alts.append((info["lam_learned"], info["u_learned"]))
            alts.append(orc.orient_multistart(Ct[i], n, st64)[:2])
        cls, det = classify_orientation(Ct[i], n, lg[i], ug[i], lo, uo, cn, alts)
        assert cls is not None, (i, det, info["beat_gap"], info["kappa_gap"])
        counts[cls] += 1
    print(f"[learned path {Bt} voxels] {counts}, fallbacks oracle {nfb} gpu {int(fb.item())}", flush=True)
    assert counts["agree"] >= 0.8 * Bt
    assert abs(int(fb.item()) - nfb) <= 2


def test_forced_fallback_equals_multistart(T, ctx):
    """kappa = +inf sends every voxel to the multistart fallback, and the merged
    answer is, exactly, the larger of the learned-only answer (kappa = -inf,
    no screening) and the plain multistart answer: the same kernels on the
    same normalised tensors, so the comparison is bit for bit."""
    n, K, B = 6, 28, 200
    rng = np.random.default_rng(9)
    C = rng.standard_normal((B, K))
    d = T.make_desc(n, 16, 7.0)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(oracle_params(10, K), K)))
    starts = cuda(synth.start_vectors())
    Cg = cuda(C.T.reshape(K, 1, 1, B))
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _, lam_m, u_m = T.extract(ctx, d, Cg, starts=starts, mlp=net, kappa=float("inf"), fallbacks=fb)
    assert int(fb.item()) == B
    _, lam_l, u_l = T.extract(ctx, d, Cg, starts=starts, mlp=net, kappa=float("-inf"), screen=False)
    _, lam_p, u_p = T.extract(ctx, d, Cg, starts=starts)
    lm, ll, lp = (x.cpu().numpy().ravel() for x in (lam_m, lam_l, lam_p))
    um, ul, up = (x.cpu().numpy().reshape(B, 3) for x in (u_m, u_l, u_p))
    plain_wins = lp > ll
    assert np.array_equal(lm, np.where(plain_wins, lp, ll))
    assert np.array_equal(um, np.where(plain_wins[:, None], up, ul))
    print(f"[forced fallback] plain larger at {int(plain_wins.sum())} of {B}", flush=True)
