"""Python binding of libttm: torch device tensors in, torch device tensors out.

Argument marshalling only -- every step runs in the HIP kernels behind the C
ABI (include/ttm.h).  Tensors must live on the context's GPU; calls are
enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from ._lib import Desc, ExtractOpts, I32x3, call, load


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libttm needs device tensors")
        if t is not None and not t.is_contiguous():
            raise ValueError("libttm needs contiguous tensors")


def n_components(degree: int, dprime: int = 3) -> int:
    return load().ttm_n_components(degree, dprime)


def spectrum_elems(fft_n: int) -> int:
    return load().ttm_spectrum_elems(fft_n)


def template_spectrum_elems(fft_n: int, L: int) -> int:
    return load().ttm_template_spectrum_elems(fft_n, L)


def make_desc(degree: int, L_edge: int, mask_radius: float, dprime: int = 3,
              filter_a: float = 0.2, eps_w: float = 1e-6, axis=(0.0, 0.0, 1.0)) -> Desc:
    d = Desc()
    d.degree, d.dprime, d.L = degree, dprime, L_edge
    d.mask_radius, d.filter_a, d.eps_w = mask_radius, filter_a, eps_w
    for i in range(3):
        d.axis[i] = axis[i]
    return d


class Context:
    """Owns a libttm context (twiddle tables) on one device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        call("ttm_create", C.byref(h), device)
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            load().ttm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ws(desc: Desc, op: int, fft_n: int, dims=(0, 0, 0), device=None) -> torch.Tensor:
    n = load().ttm_workspace_size(C.byref(desc), op, fft_n, *dims)
    if n == 0:
        raise ValueError("invalid workspace request")
    return torch.empty(n, dtype=torch.uint8, device=device)


def build_tensor(ctx: Context, desc: Desc, tmpl: torch.Tensor, quats: torch.Tensor,
                 wedge: float | None = None):
    """Tensor template T (K x L^3) and t' (L^3), Alg. 1; with ``wedge`` (the
    missing wedge's half-angle in degrees) the wedge-aware template of
    ttm_build_tensor_wedge."""
    _need_cuda(tmpl, quats)
    K = n_components(desc.degree, desc.dprime)
    Le = desc.L
    T = torch.empty((K, Le, Le, Le), dtype=torch.float32, device=tmpl.device)
    tn = torch.empty((Le, Le, Le), dtype=torch.float32, device=tmpl.device)
    if wedge is None:
        call("ttm_build_tensor", ctx.h, C.byref(desc), _ptr(tmpl), _ptr(quats), quats.shape[0],
             _ptr(T), _ptr(tn), _stream())
    else:
        ws = _ws(desc, L.TTM_OP_TENSOR_WEDGE, 0, device=tmpl.device)
        call("ttm_build_tensor_wedge", ctx.h, C.byref(desc), _ptr(tmpl), _ptr(quats),
             quats.shape[0], float(wedge), _ptr(T), _ptr(tn), _ptr(ws), ws.numel(), _stream())
    return T, tn


def template_spectra(ctx: Context, desc: Desc, T: torch.Tensor, fft_n: int) -> torch.Tensor:
    """(K + 1) x/y-transformed templates (last: mask), their L nonzero z planes:
    float32 view (K+1, L, N/2+1, N, 2); the z transform is taken per tile."""
    _need_cuda(T)
    K = n_components(desc.degree, desc.dprime)
    out = torch.empty((K + 1, desc.L, fft_n // 2 + 1, fft_n, 2), dtype=torch.float32,
                      device=T.device)
    ws = _ws(desc, L.TTM_OP_SPECTRA, fft_n, device=T.device)
    call("ttm_template_spectra", ctx.h, C.byref(desc), _ptr(T), fft_n, _ptr(out), _ptr(ws),
         ws.numel(), _stream())
    return out


def normalize(ctx: Context, desc: Desc, vol: torch.Tensor, spectra: torch.Tensor, fft_n: int,
              ws: torch.Tensor | None = None):
    """g = h*f, w (full size, 0 off the valid region), stats = (mean g, mean g^2)."""
    _need_cuda(vol, spectra)
    nz, ny, nx = vol.shape
    g = torch.empty_like(vol)
    w = torch.empty_like(vol)
    stats = torch.empty(2, dtype=torch.float64, device=vol.device)
    if ws is None:
        ws = _ws(desc, L.TTM_OP_NORMALIZE, fft_n, (nz, ny, nx), device=vol.device)
    mask_spec = spectra[-1]
    call("ttm_normalize", ctx.h, C.byref(desc), _ptr(vol), nz, ny, nx, _ptr(mask_spec), fft_n,
         _ptr(g), _ptr(w), _ptr(stats), _ptr(ws), ws.numel(), _stream())
    return g, w, stats


def prefilter(ctx: Context, desc: Desc, vol: torch.Tensor, ws: torch.Tensor | None = None):
    """g = h*f, w cleared to 0, stats = (mean g, mean g^2): the first half of normalize."""
    _need_cuda(vol)
    nz, ny, nx = vol.shape
    g = torch.empty_like(vol)
    w = torch.empty_like(vol)
    stats = torch.empty(2, dtype=torch.float64, device=vol.device)
    if ws is None:
        ws = _ws(desc, L.TTM_OP_PREFILTER, 0, (nz, ny, nx), device=vol.device)
    call("ttm_prefilter", ctx.h, C.byref(desc), _ptr(vol), nz, ny, nx, _ptr(g), _ptr(w),
         _ptr(stats), _ptr(ws), ws.numel(), _stream())
    return g, w, stats


def normalize_box(ctx: Context, desc: Desc, g: torch.Tensor, stats: torch.Tensor,
                  spectra: torch.Tensor, fft_n: int, box_lo, box_size, w: torch.Tensor,
                  ws: torch.Tensor | None = None) -> None:
    """w on one box of the valid region (the second half of normalize)."""
    _need_cuda(g, stats, spectra, w)
    nz, ny, nx = g.shape
    if ws is None:
        ws = _ws(desc, L.TTM_OP_NORMALIZE, fft_n, (nz, ny, nx), device=g.device)
    call("ttm_normalize_box", ctx.h, C.byref(desc), _ptr(g), nz, ny, nx, _ptr(stats),
         _ptr(spectra[-1]), fft_n, I32x3(*box_lo), I32x3(*box_size), _ptr(w), _ptr(ws),
         ws.numel(), _stream())


def correlate(ctx: Context, desc: Desc, g: torch.Tensor, w: torch.Tensor, stats: torch.Tensor,
              spectra: torch.Tensor, fft_n: int, box_lo, box_size, dtype=torch.float32,
              out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """C (K x bz x by x bx) on a box of the valid region (Eq. tcc / Alg. 2)."""
    _need_cuda(g, w, stats, spectra)
    nz, ny, nx = g.shape
    K = n_components(desc.degree, desc.dprime)
    if out is None:
        out = torch.empty((K, *box_size), dtype=dtype, device=g.device)
    code = L.TTM_BF16 if out.dtype == torch.bfloat16 else L.TTM_F32
    if ws is None:
        ws = _ws(desc, L.TTM_OP_CORRELATE, fft_n, (nz, ny, nx), device=g.device)
    call("ttm_correlate", ctx.h, C.byref(desc), _ptr(g), _ptr(w), nz, ny, nx, _ptr(stats),
         _ptr(spectra), fft_n, I32x3(*box_lo), I32x3(*box_size), code, _ptr(out), _ptr(ws),
         ws.numel(), _stream())
    return out


def normalize_correlate(ctx: Context, desc: Desc, g: torch.Tensor, stats: torch.Tensor,
                        spectra: torch.Tensor, fft_n: int, box_lo, box_size, w: torch.Tensor,
                        dtype=torch.float32, out: torch.Tensor | None = None,
                        ws: torch.Tensor | None = None) -> torch.Tensor:
    """normalize_box then correlate on one FFT tile, sharing the tile's forward
    transform of g: w on the box and C (K x bz x by x bx)."""
    _need_cuda(g, stats, spectra, w)
    nz, ny, nx = g.shape
    K = n_components(desc.degree, desc.dprime)
    if out is None:
        out = torch.empty((K, *box_size), dtype=dtype, device=g.device)
    code = L.TTM_BF16 if out.dtype == torch.bfloat16 else L.TTM_F32
    if ws is None:
        ws = _ws(desc, L.TTM_OP_NORM_CORR, fft_n, device=g.device)
    call("ttm_normalize_correlate", ctx.h, C.byref(desc), _ptr(g), nz, ny, nx, _ptr(stats),
         _ptr(spectra), fft_n, I32x3(*box_lo), I32x3(*box_size), _ptr(w), code, _ptr(out),
         _ptr(ws), ws.numel(), _stream())
    return out


def extract(ctx: Context, desc: Desc, Cf: torch.Tensor, *, score=None, lam=None, direction=None,
            out_lo=(0, 0, 0), out_dims=None, starts: torch.Tensor | None = None,
            orient: bool = True, max_iter: int = 500, tol: float = 1e-5, newton: int = 2,
            counters: torch.Tensor | None = None, mlp: "MLP | None" = None, kappa: float = 0.0,
            start_only: bool = False, fallbacks: torch.Tensor | None = None,
            ws: torch.Tensor | None = None, screen: bool = True, noalloc: bool = False):
    """Score / lambda / direction maps for the box held in Cf (K x bz x by x bx).

    With ``mlp`` the orientation search starts from the learned start and falls
    back to the multistart search where lambda / ||C|| < kappa or SS-HOPM did
    not converge.  ``fallbacks`` (device int32[1]) accumulates the fallback count.
    ``noalloc`` calls ttm_extract_noalloc (the library's own scratch, no
    workspace argument).
    """
    _need_cuda(Cf, score, lam, direction, starts)
    box = tuple(Cf.shape[1:])
    if out_dims is None:
        out_dims = box
    dev = Cf.device
    if score is None:
        score = torch.zeros(out_dims, dtype=torch.float32, device=dev)
    mode = L.TTM_SCORE
    opts = ExtractOpts()
    if orient:
        mode |= L.TTM_ORIENT
        if lam is None:
            lam = torch.zeros(out_dims, dtype=torch.float32, device=dev)
        if direction is None:
            direction = torch.zeros((*out_dims, desc.dprime), dtype=torch.float32, device=dev)
        if starts is None:
            raise ValueError("orientation needs start vectors")
        opts.n_starts = starts.shape[0]
        opts.starts = starts.data_ptr()
        if mlp is not None:
            mode |= L.TTM_START_MLP
            if start_only:
                mode |= L.TTM_START_ONLY
            if not screen:
                mode |= L.TTM_NO_SCREEN
            opts.mlp = mlp.packed.data_ptr()
            opts.fallback_kappa = kappa
        if ws is None and not noalloc:
            ws = _ws(desc, L.TTM_OP_EXTRACT, 0, box, device=dev)
    opts.mode = mode
    opts.max_iter = max_iter
    opts.tol = tol
    opts.newton_steps = newton
    if counters is not None:
        if counters.dtype != torch.int64 or counters.numel() < 5 or not counters.is_cuda:
            raise ValueError("counters must be a device int64 tensor of 5 elements")
        opts.work_counters = counters.data_ptr()
    code = L.TTM_BF16 if Cf.dtype == torch.bfloat16 else L.TTM_F32
    if noalloc:
        call("ttm_extract_noalloc", ctx.h, C.byref(desc), _ptr(Cf), code, I32x3(*box),
             C.byref(opts), _ptr(score), _ptr(lam) if orient else None,
             _ptr(direction) if orient else None, I32x3(*out_lo), I32x3(*out_dims),
             _ptr(fallbacks), _stream())
        return score, lam, direction
    call("ttm_extract", ctx.h, C.byref(desc), _ptr(Cf), code, I32x3(*box), C.byref(opts),
         _ptr(score), _ptr(lam) if orient else None, _ptr(direction) if orient else None,
         I32x3(*out_lo), I32x3(*out_dims), _ptr(fallbacks), _ptr(ws),
         0 if ws is None else ws.numel(), _stream())
    return score, lam, direction


def refine(ctx: Context, desc: Desc, g: torch.Tensor, w: torch.Tensor, T: torch.Tensor,
           tn: torch.Tensor, peaks: torch.Tensor, starts: torch.Tensor, r_s: float = 3.0,
           max_iter: int = 500, tol: float = 1e-5, newton: int = 2,
           ws: torch.Tensor | None = None) -> dict:
    """TTM-ref (Alg. 3) of the peaks (device int32 P x 3), quaternion form:
    refined positions, their rotations and LNCC, and the unrefined peak's own
    rotation and LNCC (TTM without refinement)."""
    _need_cuda(g, w, T, tn, peaks, starts)
    nz, ny, nx = g.shape
    P = peaks.shape[0]
    dev = g.device
    out = {"pos": torch.empty((P, 3), dtype=torch.int32, device=dev),
           "quat": torch.empty((P, 4), dtype=torch.float32, device=dev),
           "lncc": torch.empty(P, dtype=torch.float32, device=dev),
           "quat_peak": torch.empty((P, 4), dtype=torch.float32, device=dev),
           "lncc_peak": torch.empty(P, dtype=torch.float32, device=dev)}
    if ws is None:
        ws = _ws(desc, L.TTM_OP_REFINE, 0, (P, int(math.ceil(r_s)), 1), device=dev)
    opts = ExtractOpts()
    opts.mode = L.TTM_ORIENT
    opts.n_starts = starts.shape[0]
    opts.starts = starts.data_ptr()
    opts.max_iter, opts.tol, opts.newton_steps = max_iter, tol, newton
    call("ttm_refine", ctx.h, C.byref(desc), _ptr(g), _ptr(w), nz, ny, nx, _ptr(T), _ptr(tn),
         _ptr(peaks), P, float(r_s), C.byref(opts), _ptr(out["pos"]), _ptr(out["quat"]),
         _ptr(out["lncc"]), _ptr(out["quat_peak"]), _ptr(out["lncc_peak"]), _ptr(ws), ws.numel(),
         _stream())
    return out


class MLP:
    """Learned start: FP32 master parameters, Adam moments and the packed BF16 copy."""

    def __init__(self, ctx: Context, desc: Desc, params: torch.Tensor):
        lib = load()
        self.n_params = lib.ttm_mlp_param_count(C.byref(desc))
        if self.n_params == 0:
            raise ValueError(f"no learned start for d'={desc.dprime}, degree {desc.degree}")
        if params.numel() != self.n_params or params.dtype != torch.float32 or not params.is_cuda:
            raise ValueError(f"params must be {self.n_params} float32 device values")
        self.ctx, self.desc = ctx, desc
        self.params = params.contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.packed = torch.empty(lib.ttm_mlp_packed_bytes(C.byref(desc)), dtype=torch.uint8,
                                  device=params.device)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self._ws = None
        self.pack()

    def pack(self):
        call("ttm_mlp_pack", self.ctx.h, C.byref(self.desc), _ptr(self.params), _ptr(self.packed),
             _stream())

    def train_step(self, Cs: torch.Tensor, targets: torch.Tensor, lr: float,
                   grads: torch.Tensor | None = None) -> torch.Tensor:
        """One Adam step on a batch (Cs: B x K raw tensors, targets: B x d'); returns the loss."""
        _need_cuda(Cs, targets, grads)
        B = Cs.shape[0]
        if self._ws is None or self._ws.numel() < load().ttm_workspace_size(
                C.byref(self.desc), L.TTM_OP_MLP_TRAIN, 0, B, 1, 1):
            self._ws = _ws(self.desc, L.TTM_OP_MLP_TRAIN, 0, (B, 1, 1), device=Cs.device)
        if lr > 0:
            self.step += 1
        call("ttm_mlp_train_step", self.ctx.h, C.byref(self.desc), _ptr(Cs), _ptr(targets), B,
             _ptr(self.params), _ptr(self.m), _ptr(self.v), max(self.step, 1), float(lr),
             _ptr(self.packed), _ptr(self.loss), _ptr(grads), _ptr(self._ws), self._ws.numel(),
             _stream())
        return self.loss


def find_peaks(ctx: Context, score: torch.Tensor, valid_lo, valid_hi, top_p: int, min_dist: float,
               ws: torch.Tensor | None = None):
    """Greedy peaks: (positions int32 (P', 3) z,y,x; scores (P',)) on the device."""
    _need_cuda(score)
    nz, ny, nx = score.shape
    peaks = torch.empty((top_p, 3), dtype=torch.int32, device=score.device)
    vals = torch.empty(top_p, dtype=torch.float32, device=score.device)
    nf = C.c_int32(0)
    if ws is None:
        d = make_desc(2, 4, 1.0)
        ws = _ws(d, L.TTM_OP_PEAKS, 32, (nz, ny, nx), device=score.device)
    call("ttm_find_peaks", ctx.h, _ptr(score), nz, ny, nx, I32x3(*valid_lo), I32x3(*valid_hi),
         top_p, float(min_dist), _ptr(peaks), _ptr(vals), C.byref(nf), _ptr(ws), ws.numel(),
         _stream())
    return peaks[:nf.value], vals[:nf.value]


def find_peaks_async(ctx: Context, score: torch.Tensor, valid_lo, valid_hi, top_p: int,
                     min_dist: float, peaks: torch.Tensor, vals: torch.Tensor,
                     n_found: torch.Tensor, ws: torch.Tensor) -> None:
    """Find Peaks without host synchronisation (graph-capture safe); n_found stays on the device."""
    _need_cuda(score, peaks, vals, n_found, ws)
    nz, ny, nx = score.shape
    call("ttm_find_peaks_async", ctx.h, _ptr(score), nz, ny, nx, I32x3(*valid_lo),
         I32x3(*valid_hi), top_p, float(min_dist), _ptr(peaks), _ptr(vals), _ptr(n_found),
         _ptr(ws), ws.numel(), _stream())


class ExtractBatch:
    """ttm_extract over many boxes in one call: entries are dicts with C (device
    K x bz x by x bx), the maps score, lam, direction and out_lo (where the box
    sits in them).  The item table is built once on the device."""

    def __init__(self, ctx: Context, desc: Desc, entries):
        dev = entries[0]["C"].device
        self.ctx, self.desc = ctx, desc
        arr = (L.ExtractItem * len(entries))()
        first = 0
        self.dtype = entries[0]["C"].dtype
        for i, e in enumerate(entries):
            _need_cuda(e["C"], e.get("score"), e["lam"], e["direction"])
            if e["C"].dtype != self.dtype:
                raise ValueError("one field dtype per batch")
            it = arr[i]
            it.C = e["C"].data_ptr()
            it.score = e["score"].data_ptr() if e.get("score") is not None else None
            it.lam, it.dir = e["lam"].data_ptr(), e["direction"].data_ptr()
            it.first = first
            box = tuple(e["C"].shape[1:])
            for a in range(3):
                it.box[a], it.out_lo[a], it.out_dims[a] = box[a], e["out_lo"][a], e["lam"].shape[a]
            first += int(np.prod(box))
        self.table = torch.from_numpy(np.frombuffer(bytes(arr), dtype=np.uint8).copy()).to(dev)
        self.n, self.total = len(entries), first

    def workspace_bytes(self) -> int:
        return load().ttm_workspace_size(C.byref(self.desc), L.TTM_OP_EXTRACT, 0, self.total, 1, 1)

    def run(self, starts: torch.Tensor, ws: torch.Tensor, mlp: "MLP | None" = None,
            kappa: float = 0.0, fallbacks: torch.Tensor | None = None, max_iter: int = 500,
            tol: float = 1e-5, newton: int = 2, screen: bool = True, orient: bool = True) -> None:
        _need_cuda(starts, ws, fallbacks)
        opts = ExtractOpts()
        mode = L.TTM_SCORE
        if orient:
            mode |= L.TTM_ORIENT
            if mlp is not None:
                mode |= L.TTM_START_MLP
                if not screen:
                    mode |= L.TTM_NO_SCREEN
                opts.mlp = mlp.packed.data_ptr()
                opts.fallback_kappa = kappa
        opts.mode = mode
        opts.n_starts, opts.starts = starts.shape[0], starts.data_ptr()
        opts.max_iter, opts.tol, opts.newton_steps = max_iter, tol, newton
        code = L.TTM_BF16 if self.dtype == torch.bfloat16 else L.TTM_F32
        call("ttm_extract_batch", self.ctx.h, C.byref(self.desc), _ptr(self.table), self.n,
             self.total, code, C.byref(opts), _ptr(fallbacks), _ptr(ws), ws.numel(), _stream())


class PeakBatch:
    """Find Peaks over many score maps in one launch (ttm_find_peaks_batch).

    entries: dicts with score (device map), lo, hi (inclusive valid box),
    top_p, min_dist, and the outputs peaks (device int32 top_p x 3), vals
    (device float top_p), n_found (device int32 view of one element).  The
    item table and the per-item scratch are built once, on the device, so the
    launch can be captured into a graph and replayed."""

    def __init__(self, ctx: Context, entries):
        lib = load()
        dev = entries[0]["score"].device
        self.ctx = ctx
        sizes = []
        for e in entries:
            _need_cuda(e["score"], e["peaks"], e["vals"], e["n_found"])
            n = lib.ttm_peaks_batch_scratch_bytes(I32x3(*e["lo"]), I32x3(*e["hi"]))
            if n == 0:
                raise ValueError("invalid valid box")
            sizes.append((n + 255) // 256 * 256)
        self.scratch = torch.empty(sum(sizes), dtype=torch.uint8, device=dev)
        arr = (L.PeakItem * len(entries))()
        off = 0
        base = self.scratch.data_ptr()
        for i, e in enumerate(entries):
            it = arr[i]
            it.score, it.peaks, it.vals = e["score"].data_ptr(), e["peaks"].data_ptr(), e["vals"].data_ptr()
            it.n_found, it.scratch = e["n_found"].data_ptr(), base + off
            off += sizes[i]
            for a in range(3):
                it.dims[a] = e["score"].shape[a]
                it.valid_lo[a], it.valid_hi[a] = e["lo"][a], e["hi"][a]
            it.top_p, it.min_dist = int(e["top_p"]), float(e["min_dist"])
        raw = np.frombuffer(bytes(arr), dtype=np.uint8)
        self.table = torch.from_numpy(raw.copy()).to(dev)
        self.n = len(entries)
        self.max_valid = [max(e["hi"][a] - e["lo"][a] + 1 for e in entries) for a in range(3)]

    def run(self) -> None:
        call("ttm_find_peaks_batch", self.ctx.h, _ptr(self.table), self.n, I32x3(*self.max_valid),
             _stream())


def fft3d_r2c(ctx: Context, x: torch.Tensor) -> torch.Tensor:
    _need_cuda(x)
    N = x.shape[0]
    out = torch.empty((N, N // 2 + 1, N, 2), dtype=torch.float32, device=x.device)
    call("ttm_fft3d_r2c", ctx.h, _ptr(x), N, _ptr(out), _stream())
    return out


def fft3d_c2r(ctx: Context, spec: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
    """Inverse of fft3d_r2c times scale; overwrites spec."""
    _need_cuda(spec)
    N = spec.shape[0]
    x = torch.empty((N, N, N), dtype=torch.float32, device=spec.device)
    call("ttm_fft3d_c2r", ctx.h, _ptr(spec), N, float(scale), _ptr(x), _stream())
    return x


# ----------------------------------------------------------------------------
# full pass over a tomogram (tiling driver)
# ----------------------------------------------------------------------------


def valid_bounds(shape, L_edge: int):
    c = L_edge // 2
    lo = (c, c, c)
    hi = tuple(d - L_edge + c for d in shape)
    return lo, hi


def tile_boxes(shape, L_edge: int, fft_n: int):
    """Valid-region boxes of (fft_n - L + 1)^3 voxels covering the valid region."""
    lo, hi = valid_bounds(shape, L_edge)
    step = fft_n - L_edge + 1
    boxes = []
    for z in range(lo[0], hi[0] + 1, step):
        for y in range(lo[1], hi[1] + 1, step):
            for x in range(lo[2], hi[2] + 1, step):
                size = (min(step, hi[0] - z + 1), min(step, hi[1] - y + 1), min(step, hi[2] - x + 1))
                boxes.append(((z, y, x), size))
    return boxes


@dataclass
class PassResult:
    score: torch.Tensor
    lam: torch.Tensor | None
    direction: torch.Tensor | None
    peaks: torch.Tensor | None
    peak_vals: torch.Tensor | None
    w: torch.Tensor
    g: torch.Tensor


class Engine:
    """A TTM full pass with preallocated buffers: prefilter, then per tile the
    local normalisation and correlation (side stream, one tile ahead) and the
    extraction into the volume maps, then Find Peaks."""

    def __init__(self, ctx: Context, desc: Desc, spectra: torch.Tensor, fft_n: int, shape,
                 starts: torch.Tensor | None, field_dtype=torch.float32, orient: bool = True,
                 max_iter: int = 500, tol: float = 1e-5, newton: int = 2,
                 mlp: MLP | None = None, kappa: float = 0.0, screen: bool = True):
        self.ctx, self.desc, self.spectra, self.fft_n = ctx, desc, spectra, fft_n
        self.shape = tuple(shape)
        self.starts, self.orient = starts, orient
        self.max_iter, self.tol, self.newton = max_iter, tol, newton
        self.mlp, self.kappa, self.screen = mlp, kappa, screen
        dev = spectra.device
        nz, ny, nx = self.shape
        K = n_components(desc.degree, desc.dprime)
        self.boxes = tile_boxes(self.shape, desc.L, fft_n)
        step = fft_n - desc.L + 1
        self.K = K
        # two tile buffers: the correlation of tile k+1 runs on a side stream
        # while tile k is extracted on the caller's stream
        self.Cbufs = [torch.empty(K * step ** 3, dtype=field_dtype, device=dev) for _ in range(2)]
        self.Cbuf = self.Cbufs[0]
        self.side = torch.cuda.Stream(device=dev)
        self.ws_pre = _ws(desc, L.TTM_OP_PREFILTER, 0, self.shape, device=dev)
        self.ws_norm = _ws(desc, L.TTM_OP_NORMALIZE, fft_n, self.shape, device=dev)
        self.ws_nc = _ws(desc, L.TTM_OP_NORM_CORR, fft_n, device=dev)
        self.ws_peaks = _ws(desc, L.TTM_OP_PEAKS, fft_n, self.shape, device=dev)
        self.ws_extract = _ws(desc, L.TTM_OP_EXTRACT, 0, (step, step, step), device=dev)
        self.fallbacks = torch.zeros(1, dtype=torch.int32, device=dev)
        self.score = torch.zeros(self.shape, dtype=torch.float32, device=dev)
        self.lam = torch.zeros(self.shape, dtype=torch.float32, device=dev) if orient else None
        self.dir = (torch.zeros((*self.shape, desc.dprime), dtype=torch.float32, device=dev)
                    if orient else None)

    def release(self) -> None:
        """Free the tile buffers and workspaces and keep the output maps (score,
        lam, dir); run() cannot be called afterwards."""
        self.Cbufs = self.Cbuf = None
        self.ws_pre = self.ws_norm = self.ws_corr = self.ws_peaks = self.ws_extract = None

    def run(self, vol: torch.Tensor, top_p: int | None = None, min_dist: float | None = None,
            tiles=None, overlap: bool = True, timing: dict | None = None,
            counters: torch.Tensor | None = None) -> PassResult:
        """One full pass.  With ``overlap`` the correlations run one tile ahead on a
        side stream (HBM-bound) under the extractions (ALU-bound).  ``timing``, if
        given, receives lists of (start, end) events per stage."""
        main = torch.cuda.current_stream()
        side = self.side if overlap else main

        def ev():
            return torch.cuda.Event(enable_timing=True) if timing is not None else None

        def rec(e, stream):
            if e is not None:
                e.record(stream)

        if timing is not None:
            for k in ("normalize", "correlate", "extract", "peaks"):
                timing.setdefault(k, [])
        e0, e1 = ev(), ev()
        rec(e0, main)
        g, w, stats = prefilter(self.ctx, self.desc, vol, ws=self.ws_pre)
        rec(e1, main)
        if timing is not None:
            timing["normalize"].append((e0, e1))
        boxes = self.boxes if tiles is None else tiles
        if overlap:
            side.wait_stream(main)
        free = [None, None]
        for k, (lo, size) in enumerate(boxes):
            b = k % 2
            Ct = self.Cbufs[b][: self.K * size[0] * size[1] * size[2]].view(self.K, *size)
            with torch.cuda.stream(side):
                # the tile's local normalisation (Eq. norm_f) and its correlation
                # share the forward transform of the tile of g
                if free[b] is not None:
                    side.wait_event(free[b])
                a0, a1 = ev(), ev()
                rec(a0, side)
                normalize_correlate(self.ctx, self.desc, g, stats, self.spectra, self.fft_n, lo,
                                    size, w, out=Ct, ws=self.ws_nc)
                rec(a1, side)
                ready = torch.cuda.Event()
                ready.record(side)
            if timing is not None:
                timing["correlate"].append((a0, a1, size))
            main.wait_event(ready)
            x0, x1 = ev(), ev()
            rec(x0, main)
            extract(self.ctx, self.desc, Ct, score=self.score, lam=self.lam, direction=self.dir,
                    out_lo=lo, out_dims=self.shape, starts=self.starts, orient=self.orient,
                    max_iter=self.max_iter, tol=self.tol, newton=self.newton, mlp=self.mlp,
                    kappa=self.kappa, fallbacks=self.fallbacks, ws=self.ws_extract,
                    screen=self.screen, counters=counters)
            rec(x1, main)
            if timing is not None:
                timing["extract"].append((x0, x1, size))
            free[b] = torch.cuda.Event()
            free[b].record(main)
        if overlap:
            main.wait_stream(side)
        peaks = vals = None
        if top_p:
            p0, p1 = ev(), ev()
            rec(p0, main)
            vlo, vhi = valid_bounds(self.shape, self.desc.L)
            peaks, vals = find_peaks(self.ctx, self.score, vlo, vhi, top_p,
                                     2.0 * self.desc.mask_radius if min_dist is None else min_dist,
                                     ws=self.ws_peaks)
            rec(p1, main)
            if timing is not None:
                timing["peaks"].append((p0, p1))
        return PassResult(self.score, self.lam, self.dir, peaks, vals, w, g)


# ----------------------------------------------------------------------------
# batches of uneven subtomograms and several templates (one graph launch)
# ----------------------------------------------------------------------------

FFT_EDGES = (64, 96, 128, 160, 192, 256, 512)


def tiles_for(shape, L_edge: int, fft_n: int) -> int:
    step = fft_n - L_edge + 1
    if step < 1:
        return 0
    return int(np.prod([-(-(d - L_edge + 1) // step) for d in shape]))


def pick_fft(shape, L_edge: int, cost: dict | None = None) -> int:
    """FFT edge of least modelled cost: tiles(N) x cost(N); cost defaults to
    N^3 log2 N; with a measured cost only the measured edges compete."""
    best, best_c = None, None
    for N in FFT_EDGES:
        t = tiles_for(shape, L_edge, N)
        if t == 0 or (cost and N not in cost):
            continue
        c = t * (cost[N] if cost else N ** 3 * np.log2(N))
        if best_c is None or c < best_c:
            best, best_c = N, c
    if best is None:
        raise ValueError("no supported FFT edge fits the template")
    return best


def deal_items(costs, branches: int) -> list:
    """Items dealt out to at most ``branches`` branches (never more branches
    than items, at least one): largest cost first, each to the branch with the
    least cost so far (the lowest-numbered one on ties).  Returns the item
    indices of each branch in the order they were dealt."""
    if branches < 1:
        raise ValueError("branches must be at least 1")
    nb = max(1, min(branches, len(costs)))
    out = [[] for _ in range(nb)]
    load_b = [0.0] * nb
    for i in sorted(range(len(costs)), key=lambda j: -costs[j]):
        b = min(range(nb), key=lambda k: load_b[k])
        out[b].append(i)
        load_b[b] += costs[i]
    return out


class BatchEngine:
    """Full TTM passes over many subtomograms of uneven size with several
    templates, recorded once into a HIP graph and replayed with one launch.

    templates: list of (desc, T) with T the K x L^3 tensor template;
    shapes: per-item volume shape; owner: per-item template index.
    Inputs are copied into ``self.volumes[i]`` before ``replay()``; outputs are
    ``score[i]``, ``lam[i]``, ``direction[i]``, ``peaks[i]``, ``vals[i]`` and
    ``n_found[i]`` (device).  ``cost`` maps FFT edge -> measured cost of one tile
    (see ``autotune``); without it the edge is chosen by N^3 log N.

    The items' normalisation and correlation chains are independent, and one
    small tile does not fill the GPU, so they are recorded on ``branches``
    streams (items dealt out by modelled cost, largest first, each to the
    least loaded branch, every branch with its own workspaces): the graph holds
    them as parallel branches.  The extractions follow once every branch is
    done (letting a template's extraction overlap the next template's
    correlations was slower: the persistent extraction kernels hold the CUs),
    one branch per template, each with its own workspace, so one template's
    small list kernels overlap another's pooled runs; then Find Peaks.  The
    outputs do not depend on the branch count.
    """

    def __init__(self, ctx: Context, templates, shapes, owner, starts: torch.Tensor, top_p: int,
                 mlps=None, kappa: float = 0.0, field_dtype=torch.float32, cost: dict | None = None,
                 orient: bool = True, branches: int = 8):
        self.ctx, self.templates, self.shapes, self.owner = ctx, templates, [tuple(s) for s in shapes], owner
        self.starts, self.top_p, self.mlps, self.kappa = starts, top_p, mlps, kappa
        self.orient, self.field_dtype = orient, field_dtype
        dev = starts.device
        self.fft = [pick_fft(s, templates[o][0].L, cost) for s, o in zip(self.shapes, owner)]
        self.spectra = {}
        for i, (s, o) in enumerate(zip(self.shapes, owner)):
            key = (o, self.fft[i])
            if key not in self.spectra:
                d, T = templates[o]
                self.spectra[key] = template_spectra(ctx, d, T, self.fft[i])
        self.volumes = [torch.zeros(s, dtype=torch.float32, device=dev) for s in self.shapes]
        self.score = [torch.zeros(s, dtype=torch.float32, device=dev) for s in self.shapes]
        self.lam = [torch.zeros(s, dtype=torch.float32, device=dev) for s in self.shapes]
        self.direction = [torch.zeros((*s, templates[o][0].dprime), dtype=torch.float32, device=dev)
                          for s, o in zip(self.shapes, owner)]
        self.peaks = [torch.zeros((top_p, 3), dtype=torch.int32, device=dev) for _ in self.shapes]
        self.vals = [torch.zeros(top_p, dtype=torch.float32, device=dev) for _ in self.shapes]
        self.n_found = torch.zeros(len(self.shapes), dtype=torch.int32, device=dev)
        self.fallbacks = torch.zeros(1, dtype=torch.int32, device=dev)
        # shared workspaces, each sized for the largest request of its kind
        ws_norm = ws_corr = 0
        lib = load()
        for s, o, N in zip(self.shapes, owner, self.fft):
            d = templates[o][0]
            ws_norm = max(ws_norm, lib.ttm_workspace_size(C.byref(d), L.TTM_OP_NORMALIZE, N, *s))
            ws_corr = max(ws_corr, lib.ttm_workspace_size(C.byref(d), L.TTM_OP_CORRELATE, N, *s))
        item_cost = [tiles_for(s, templates[o][0].L, N) * (cost[N] if cost else N ** 3 * np.log2(N))
                     for s, o, N in zip(self.shapes, owner, self.fft)]
        self.branch_items = deal_items(item_cost, branches)
        self.branches = len(self.branch_items)
        self.ws_norm = [torch.empty(ws_norm, dtype=torch.uint8, device=dev) for _ in range(self.branches)]
        self.ws_corr = [torch.empty(ws_corr, dtype=torch.uint8, device=dev) for _ in range(self.branches)]
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(self.branches)]
        # each item's field in its own slice of its template's buffer, so that one
        # extraction call serves every item of a template
        self.groups = sorted(set(owner))
        self.Cslice = [None] * len(self.shapes)
        self.extract_batches = {}
        self.Cgroup = {}

        for o in self.groups:
            d = templates[o][0]
            K = n_components(d.degree, d.dprime)
            idx = [i for i in range(len(self.shapes)) if owner[i] == o]
            sizes = []
            for i in idx:
                lo, hi = valid_bounds(self.shapes[i], d.L)
                sizes.append(tuple(h - l + 1 for l, h in zip(lo, hi)))
            total = sum(int(np.prod(sz)) for sz in sizes)
            buf = torch.empty(K * total, dtype=field_dtype, device=dev)
            self.Cgroup[o] = buf
            off = 0
            entries = []
            for i, sz in zip(idx, sizes):
                nv = int(np.prod(sz))
                self.Cslice[i] = buf[K * off: K * (off + nv)].view(K, *sz)
                off += nv
                lo, _ = valid_bounds(self.shapes[i], d.L)
                entries.append(dict(C=self.Cslice[i], score=self.score[i], lam=self.lam[i],
                                    direction=self.direction[i], out_lo=lo))
            eb = ExtractBatch(ctx, d, entries)
            self.extract_batches[o] = eb
        # each template's extraction on a branch of its own, with its own workspace
        self.ws_ext = {o: torch.empty(self.extract_batches[o].workspace_bytes(), dtype=torch.uint8,
                                      device=dev) for o in self.groups}
        self.ext_streams = {o: torch.cuda.Stream(device=dev) for o in self.groups}
        # Find Peaks of every item in one launch
        entries = []
        for i, (s, o) in enumerate(zip(self.shapes, owner)):
            d = templates[o][0]
            lo, hi = valid_bounds(s, d.L)
            entries.append(dict(score=self.score[i], lo=lo, hi=hi, top_p=top_p,
                                min_dist=2.0 * d.mask_radius, peaks=self.peaks[i], vals=self.vals[i],
                                n_found=self.n_found[i:i + 1]))
        self.peak_batch = PeakBatch(ctx, entries)
        self.g = [torch.empty(s, dtype=torch.float32, device=dev) for s in self.shapes]
        self.w = [torch.empty(s, dtype=torch.float32, device=dev) for s in self.shapes]
        self.stats = torch.zeros((len(self.shapes), 2), dtype=torch.float64, device=dev)
        self.graph = None

    def _correlate_item(self, i, b):
        """Item i's normalisation and correlation on the current stream with
        branch b's workspaces."""
        o = self.owner[i]
        d = self.templates[o][0]
        N = self.fft[i]
        nz, ny, nx = self.shapes[i]
        spec = self.spectra[(o, N)]
        call("ttm_normalize", self.ctx.h, C.byref(d), _ptr(self.volumes[i]), nz, ny, nx,
             _ptr(spec[-1]), N, _ptr(self.g[i]), _ptr(self.w[i]), _ptr(self.stats[i]),
             _ptr(self.ws_norm[b]), self.ws_norm[b].numel(), _stream())
        lo, hi = valid_bounds(self.shapes[i], d.L)
        size = tuple(h - l + 1 for l, h in zip(lo, hi))
        correlate(self.ctx, d, self.g[i], self.w[i], self.stats[i], spec, N, lo, size,
                  out=self.Cslice[i], ws=self.ws_corr[b])

    def run_eager(self):
        """The whole batch, ordered after the current stream's earlier work and
        before its later work (also what the graph records): each item's
        normalisation and correlation into its slice of its template's field
        buffer on its branch, then one extraction per template (each on its
        own branch), then one Find Peaks launch for every item."""
        main = torch.cuda.current_stream()
        for b, st in enumerate(self.streams):
            st.wait_stream(main)
            with torch.cuda.stream(st):
                for i in self.branch_items[b]:
                    self._correlate_item(i, b)
        for st in self.streams:
            main.wait_stream(st)
        for o in self.groups:
            st = self.ext_streams[o]
            st.wait_stream(main)
            with torch.cuda.stream(st):
                mlp = self.mlps[o] if self.mlps is not None else None
                self.extract_batches[o].run(self.starts, self.ws_ext[o], mlp=mlp, kappa=self.kappa,
                                            fallbacks=self.fallbacks, orient=self.orient)
        for o in self.groups:
            main.wait_stream(self.ext_streams[o])
        self.peak_batch.run()

    def capture(self):
        """Record the whole batch into one HIP graph (after a warm-up on a side stream)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run_eager()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run_eager()
        torch.cuda.synchronize()

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()


def autotune(ctx: Context, desc: Desc, edges=FFT_EDGES, reps: int = 3) -> dict:
    """Measured cost (ms) of one full-tile correlation per FFT edge (normalisation excluded)."""
    cost = {}
    dev = torch.device("cuda", ctx.device)
    K = n_components(desc.degree, desc.dprime)
    for N in edges:
        if N < desc.L:
            continue
        T = torch.zeros((K, desc.L, desc.L, desc.L), dtype=torch.float32, device=dev)
        spec = template_spectra(ctx, desc, T, N)
        vol = torch.randn((N, N, N), dtype=torch.float32, device=dev)
        g, w, stats = normalize(ctx, desc, vol, spec, N)
        lo, hi = valid_bounds(vol.shape, desc.L)
        size = tuple(h - l + 1 for l, h in zip(lo, hi))
        out = torch.empty((K, *size), dtype=torch.float32, device=dev)
        ws = _ws(desc, L.TTM_OP_CORRELATE, N, vol.shape, device=dev)
        correlate(ctx, desc, g, w, stats, spec, N, lo, size, out=out, ws=ws)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            correlate(ctx, desc, g, w, stats, spec, N, lo, size, out=out, ws=ws)
        b.record()
        torch.cuda.synchronize()
        cost[N] = a.elapsed_time(b) / reps
        del T, spec, vol, g, w, out, ws
    return cost
