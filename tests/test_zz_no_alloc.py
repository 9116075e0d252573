"""ttm_extract_noalloc (the library's own device scratch, no workspace
argument) against ttm_extract (a caller workspace): the same kernels on the
same inputs, so the outputs must be identical, bit for bit.  Two calls in a
row, the second on a smaller box, so a stale scratch from the first call
would show; then a box too large for the scratch must be rejected before
anything runs."""
import numpy as np
import pytest

import synth
from tests.gpu_common import oracle_trained_params, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def test_noalloc_extract_equals_extract_on_two_calls():
    require_gpu()
    from oracle import mlp as omlp
    from oracle import sym
    from paper_2408_02398_amd import ttm
    from paper_2408_02398_amd._lib import TTMError
    ctx = ttm.Context(0)
    n, K = 6, 28
    d = ttm.make_desc(n, 16, 7.0)
    pl = oracle_trained_params(12, n)
    net = ttm.MLP(ctx, d, cuda(omlp.pad_params(pl, K)))
    starts = cuda(synth.start_vectors())
    rng = np.random.default_rng(31)
    for box in [(30, 33, 37), (9, 11, 13)]:
        print(f"[noalloc] box {box}", flush=True)
        vs = rng.standard_normal((int(np.prod(box)), 3))
        vs /= np.linalg.norm(vs, axis=1, keepdims=True)
        C = (sym.monomials(vs, n) + 0.3 * rng.standard_normal((len(vs), K))).T.reshape(K, *box)
        Cg = cuda(C)
        for mlp in (None, net):
            outs = []
            for noalloc in (False, True):
                fb = torch.zeros(1, dtype=torch.int32, device="cuda")
                s, lam, u = ttm.extract(ctx, d, Cg, starts=starts, mlp=mlp, kappa=0.3,
                                        fallbacks=fb, noalloc=noalloc)
                torch.cuda.synchronize()
                outs.append((s.clone(), lam.clone(), u.clone(), int(fb.item())))
            a, b = outs
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
            assert a[3] == b[3]
    # a box whose scratch exceeds the library's array is refused on the host
    big = torch.zeros((K, 200, 200, 200), dtype=torch.float32, device="cuda")
    with pytest.raises(TTMError):
        ttm.extract(ctx, d, big, starts=starts, noalloc=True)
