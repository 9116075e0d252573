"""ctypes declarations of the libttm C ABI (include/ttm.h).

The shared library is built in-tree by ``paper_2408_02398_amd.build``.  There
is no fallback: if libttm.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttm.so")

TTM_OK, TTM_EINVAL, TTM_ENOMEM, TTM_EDEVICE, TTM_EUNSUPPORTED, TTM_EWORKSPACE = 0, -1, -2, -3, -4, -5
TTM_F32, TTM_BF16 = 0, 1
TTM_OP_SPECTRA, TTM_OP_NORMALIZE, TTM_OP_CORRELATE, TTM_OP_PEAKS = 1, 2, 3, 4
TTM_SCORE, TTM_ORIENT, TTM_START_MLP, TTM_START_ONLY, TTM_NO_SCREEN = 1, 2, 4, 8, 16
TTM_OP_EXTRACT, TTM_OP_MLP_TRAIN, TTM_OP_PREFILTER, TTM_OP_REFINE = 5, 6, 7, 8
TTM_OP_TENSOR_WEDGE, TTM_OP_NORM_CORR = 9, 10

STATUS_NAMES = {0: "TTM_OK", -1: "TTM_EINVAL", -2: "TTM_ENOMEM", -3: "TTM_EDEVICE",
                -4: "TTM_EUNSUPPORTED", -5: "TTM_EWORKSPACE"}


class Desc(C.Structure):
    _fields_ = [("degree", C.c_int32), ("dprime", C.c_int32), ("L", C.c_int32),
                ("mask_radius", C.c_float), ("filter_a", C.c_float), ("eps_w", C.c_float),
                ("axis", C.c_float * 3)]


class ExtractOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_starts", C.c_int32), ("starts", C.c_void_p),
                ("mlp", C.c_void_p), ("fallback_kappa", C.c_float), ("max_iter", C.c_int32),
                ("tol", C.c_float), ("newton_steps", C.c_int32), ("work_counters", C.c_void_p)]


class PeakItem(C.Structure):
    _fields_ = [("score", C.c_void_p), ("peaks", C.c_void_p), ("vals", C.c_void_p),
                ("n_found", C.c_void_p), ("scratch", C.c_void_p), ("dims", C.c_int32 * 3),
                ("valid_lo", C.c_int32 * 3), ("valid_hi", C.c_int32 * 3), ("top_p", C.c_int32),
                ("min_dist", C.c_float)]


class ExtractItem(C.Structure):
    _fields_ = [("C", C.c_void_p), ("score", C.c_void_p), ("lam", C.c_void_p), ("dir", C.c_void_p),
                ("first", C.c_uint64), ("box", C.c_int32 * 3), ("out_lo", C.c_int32 * 3),
                ("out_dims", C.c_int32 * 3), ("reserved", C.c_int32)]


I32x3 = C.c_int32 * 3
vp = C.c_void_p
DP = C.POINTER(Desc)

# name -> (restype, argtypes)
SIGNATURES = {
    "ttm_create": (C.c_int, [C.POINTER(vp), C.c_int]),
    "ttm_destroy": (None, [vp]),
    "ttm_last_error": (C.c_char_p, []),
    "ttm_n_components": (C.c_int, [C.c_int, C.c_int]),
    "ttm_spectrum_elems": (C.c_size_t, [C.c_int]),
    "ttm_template_spectrum_elems": (C.c_size_t, [C.c_int, C.c_int]),
    "ttm_fft_supported": (C.c_int, [C.c_int]),
    "ttm_workspace_size": (C.c_size_t, [DP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "ttm_build_tensor": (C.c_int, [vp, DP, vp, vp, C.c_int, vp, vp, vp]),
    "ttm_build_tensor_wedge": (C.c_int, [vp, DP, vp, vp, C.c_int, C.c_float, vp, vp, vp, C.c_size_t,
                                         vp]),
    "ttm_template_spectra": (C.c_int, [vp, DP, vp, C.c_int, vp, vp, C.c_size_t, vp]),
    "ttm_normalize": (C.c_int, [vp, DP, vp, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp, vp, vp,
                                vp, C.c_size_t, vp]),
    "ttm_prefilter": (C.c_int, [vp, DP, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp,
                                C.c_size_t, vp]),
    "ttm_normalize_box": (C.c_int, [vp, DP, vp, C.c_int, C.c_int, C.c_int, vp, vp, C.c_int,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp, vp, C.c_size_t,
                                    vp]),
    "ttm_correlate": (C.c_int, [vp, DP, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, C.c_int,
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int, vp, vp,
                                C.c_size_t, vp]),
    "ttm_normalize_correlate": (C.c_int, [vp, DP, vp, C.c_int, C.c_int, C.c_int, vp, vp, C.c_int,
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp, C.c_int, vp,
                                          vp, C.c_size_t, vp]),
    "ttm_extract": (C.c_int, [vp, DP, vp, C.c_int, C.POINTER(C.c_int32), C.POINTER(ExtractOpts),
                              vp, vp, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp, vp,
                              C.c_size_t, vp]),
    "ttm_extract_noalloc": (C.c_int, [vp, DP, vp, C.c_int, C.POINTER(C.c_int32),
                                      C.POINTER(ExtractOpts), vp, vp, vp, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), vp, vp]),
    "ttm_refine": (C.c_int, [vp, DP, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, C.c_int,
                             C.c_float, C.POINTER(ExtractOpts), vp, vp, vp, vp, vp, vp, C.c_size_t,
                             vp]),
    "ttm_extract_batch": (C.c_int, [vp, DP, vp, C.c_int, C.c_uint64, C.c_int, C.POINTER(ExtractOpts),
                                    vp, vp, C.c_size_t, vp]),
    "ttm_mlp_param_count": (C.c_size_t, [DP]),
    "ttm_mlp_packed_bytes": (C.c_size_t, [DP]),
    "ttm_mlp_pack": (C.c_int, [vp, DP, vp, vp, vp]),
    "ttm_mlp_train_step": (C.c_int, [vp, DP, vp, vp, C.c_int, vp, vp, vp, C.c_int, C.c_float, vp,
                                     vp, vp, vp, C.c_size_t, vp]),
    "ttm_find_peaks": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.c_int, C.c_float, vp, vp,
                                 C.POINTER(C.c_int32), vp, C.c_size_t, vp]),
    "ttm_find_peaks_async": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.c_int, C.c_float, vp, vp, vp, vp,
                                       C.c_size_t, vp]),
    "ttm_peaks_batch_scratch_bytes": (C.c_size_t, [C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ttm_find_peaks_batch": (C.c_int, [vp, vp, C.c_int, C.POINTER(C.c_int32), vp]),
    "ttm_fft3d_r2c": (C.c_int, [vp, vp, C.c_int, vp, vp]),
    "ttm_fft3d_c2r": (C.c_int, [vp, vp, C.c_int, C.c_float, vp, vp]),
}

_lock = threading.Lock()
_lib = None


class TTMError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libttm.so and declare its signatures (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(
                    f"libttm.so not found at {path}: build it with "
                    "`python -m paper_2408_02398_amd.build` (no CPU fallback exists)")
            lib = C.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def check(fn: str, code: int) -> None:
    if code != TTM_OK:
        msg = load().ttm_last_error()
        raise TTMError(fn, code, msg.decode() if msg else "")


def call(fn: str, *args) -> None:
    check(fn, getattr(load(), fn)(*args))
