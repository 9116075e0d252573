"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2408_02398_amd", "libttm.so")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    if not os.path.exists(LIB):
        pytest.fail("libttm.so is not built: the GPU path has no fallback")


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def oracle_trained_params(seed: int, n: int, steps: int = 300, batch: int = 2048,
                          noise: float = 0.15, lr: float = 3e-3):
    """Learned-start network parameters trained by the FP64 oracle on the CPU.

    Training tensors are rank-one tensors v^n of random unit directions plus
    Gaussian noise, with v as the target.  Both sides of a parity test consume
    these parameters, so no input of the oracle comes from the GPU path.
    """
    from oracle import mlp as omlp
    from oracle import sym
    rng = np.random.default_rng(seed)
    K = sym.n_components(n, 3)
    p = omlp.init_params(rng, K)
    st = omlp.adam_init(p)
    for _ in range(steps):
        v = rng.standard_normal((batch, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        C = sym.monomials(v, n) + noise * rng.standard_normal((batch, K))
        _, cache = omlp.forward(p, omlp.features(C, n))
        omlp.adam_step(p, omlp.backward(p, cache, v), st, lr=lr)
    return p
