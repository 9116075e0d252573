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
                          noise: float = 0.15, lr: float = 3e-3, d: int = 3):
    """Learned-start network parameters trained by the FP64 oracle on the CPU.

    Training tensors are rank-one tensors v^n of random unit vectors of R^d
    (axes, or quaternions at d = 4) plus Gaussian noise, with v as the target.
    Both sides of a parity test consume these parameters, so no input of the
    oracle comes from the GPU path.
    """
    from oracle import mlp as omlp
    from oracle import sym
    rng = np.random.default_rng(seed)
    K = sym.n_components(n, d)
    p = omlp.init_params(rng, K, d_out=d)
    st = omlp.adam_init(p)
    for _ in range(steps):
        v = rng.standard_normal((batch, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        C = sym.monomials(v, n) + noise * rng.standard_normal((batch, K))
        _, cache = omlp.forward(p, omlp.features(C, n, d))
        omlp.adam_step(p, omlp.backward(p, cache, v), st, lr=lr)
    return p


def classify_orientation(Cv, n, lam_g, u_g, lam_o, u_o, floor, alts=()):
    """Class of one GPU orientation (lambda_g, u_g) against the oracle's
    converged answer (lambda_o, u_o) for the FP64 tensor Cv (Sec. 3.1):

    'agree'  u_g within 1 degree of u_o, lambda_g within 1e-4 floor of lambda_o;
    'near'   the GPU found a maximiser of the FP64 function as good as the
             oracle's up to the score tolerance, on a flat maximum or one of two
             tied maxima, where the FP32 field (which differs from the FP64 one by
             rounding) moves the maximiser by more than 1 degree:
             lambda_g and <C, u_g^n> are both within 1e-4 floor of lambda_o, and
             the converged ascent from u_g reaches a maximum within 1e-4 floor
             of lambda_o;
    'alt'    the same, against one of the answers in ``alts`` ((lambda, u)
             pairs the method may give; e.g. from starts tilted by rounding);
    None     unclassified: a parity failure.
    Returns (class, details dict).
    """
    from oracle import sym
    from oracle import ttm as orc
    d = len(u_o)
    tol = 1e-4 * floor
    ang = float(orc.axis_distance_deg(u_g, u_o)) if np.linalg.norm(u_g) > 0 else 180.0
    info = {"angle": ang, "dlam": float(lam_g - lam_o)}
    if ang < 1.0 and abs(lam_g - lam_o) <= tol:
        return "agree", info
    cn = float(sym.frobenius(Cv, n, d))
    if cn == 0.0 or not np.linalg.norm(u_g) > 0:
        return None, info
    Cu = np.asarray(Cv, dtype=np.float64) / cn
    ug = np.asarray(u_g, dtype=np.float64) / np.linalg.norm(u_g)
    f_g = cn * float(sym.inner_power(Cu, ug, n))
    lam_a, u_a, _ = orc.converge(Cu, n, ug, orc.unfolding_shift(Cu, n, d))
    lam_a *= cn
    info.update({"f64_at_gpu_u": f_g, "ascent_lam": lam_a,
                 "ascent_moved_deg": float(orc.axis_distance_deg(u_a, ug))})
    for name, targets in (("near", [(lam_o, u_o)]), ("alt", list(alts))):
        for lam_t, _ in targets:
            if (abs(lam_g - lam_t) <= tol and abs(f_g - lam_t) <= tol and abs(lam_a - lam_t) <= tol):
                return name, info
    return None, info
