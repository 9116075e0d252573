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
from tests.gpu_common import oracle_trained_params, require_gpu

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
    for i in range(Bt):
        lo, uo, fell = omlp.orient_learned(Ct[i], n, pl, starts.astype(np.float64), kappa)
        nfb += fell
        assert abs(lg[i] - lo) <= 1e-4 * max(orc.score(Ct[i], n), 1e-9)
        if orc.sshopm_rate(Ct[i], n, uo) < 0.95:
            assert orc.angle_deg(ug[i], uo) < 1.0
    assert abs(int(fb.item()) - nfb) <= 2


def test_forced_fallback_equals_multistart(T, ctx):
    n, K, B = 6, 28, 200
    rng = np.random.default_rng(9)
    C = rng.standard_normal((B, K))
    d = T.make_desc(n, 16, 7.0)
    net = T.MLP(ctx, d, cuda(omlp.pad_params(oracle_params(10, K), K)))
    starts = cuda(synth.start_vectors())
    Cg = cuda(C.T.reshape(K, 1, 1, B))
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _, lam_l, u_l = T.extract(ctx, d, Cg, starts=starts, mlp=net, kappa=float("inf"), fallbacks=fb)
    _, lam_p, u_p = T.extract(ctx, d, Cg, starts=starts)
    assert int(fb.item()) == B
    ll, lp = lam_l.cpu().numpy().ravel(), lam_p.cpu().numpy().ravel()
    # every voxel fell back, so the answer is the larger of the learned one and
    # the multistart's, which is the plain multistart computed by the same kernels
    assert np.all(ll >= lp)
    eq = ll == lp
    assert eq.mean() > 0.5
    # equal lambda: the multistart answer, or the learned one at the same maximum
    # (lambda is flat there, so FP32 lambda ties while u differs by rounding)
    ang = orc.angle_deg(u_l.cpu().numpy().reshape(B, 3)[eq], u_p.cpu().numpy().reshape(B, 3)[eq])
    assert np.max(ang) < 0.1

