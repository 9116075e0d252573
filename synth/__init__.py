"""Seeded synthetic inputs for tensorial template matching (TTM).

This module only *generates inputs*: Gaussian-blob templates, tomograms holding
rotated copies of a template plus noise and a missing wedge, rotation sample
sets for the SO(3) integral, and the fixed start vectors of the multi-start
orientation search.  It holds none of the matching arithmetic (filtering,
normalisation, tensor construction, correlation, extraction, peak picking):
both the CPU oracle (through the tests) and the GPU path consume what it
produces, and neither imports the other.

Workload recipes follow the paper's synthetic experiments in spirit (Sec. 4.1:
randomly rotated copies of one template in a tomogram, additive Gaussian noise
at a stated SNR) with Gaussian-blob templates standing in for the PDB-derived
densities and the EMPIAR-10988 tomogram, which are not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# rotations (input generation only: random poses of copies and blob axes)
# --------------------------------------------------------------------------


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices from unit quaternions (w, x, y, z), Hamilton product."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-uniform unit quaternions (normalised 4D Gaussians), w >= 0."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    return _quat_to_rot(random_quaternions(rng, n))


# --------------------------------------------------------------------------
# SO(3) sample sets for the rotation integral of the tensor template
# --------------------------------------------------------------------------

# psi is the real root of psi^4 = psi + 4 used by super-Fibonacci spirals
# (Alexa 2022, "Super-Fibonacci spirals: fast, low-discrepancy sampling of SO(3)").
_PSI = 1.533751168755204288118041
_PHI = math.sqrt(2.0)


def super_fibonacci(n: int) -> np.ndarray:
    """n unit quaternions (w, x, y, z) of the super-Fibonacci spiral on S^3."""
    s = np.arange(n, dtype=np.float64) + 0.5
    r = np.sqrt(s / n)
    big_r = np.sqrt(1.0 - s / n)
    alpha = 2.0 * np.pi * s / _PHI
    beta = 2.0 * np.pi * s / _PSI
    return np.stack([r * np.sin(alpha), r * np.cos(alpha),
                     big_r * np.sin(beta), big_r * np.cos(beta)], axis=1)


def octahedral_quaternions() -> np.ndarray:
    """The 24 rotations of the cube (grid-preserving rotations) as unit quaternions."""
    h = 1.0 / math.sqrt(2.0)
    qs = [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)]
    for ax in range(3):                       # +-90 degrees about each axis
        for sgn in (1, -1):
            q = [h, 0, 0, 0]
            q[1 + ax] = sgn * h
            qs.append(tuple(q))
    for a, b in ((1, 2), (1, 3), (2, 3)):     # 180 degrees about face diagonals
        for sgn in (1, -1):
            q = [0, 0, 0, 0]
            q[a] = h
            q[b] = sgn * h
            qs.append(tuple(q))
    for sx in (1, -1):                        # 120 degrees about body diagonals
        for sy in (1, -1):
            for sz in (1, -1):
                qs.append((0.5, 0.5 * sx, 0.5 * sy, 0.5 * sz))
    out = np.array(qs, dtype=np.float64)
    assert out.shape == (24, 4)
    return out


def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def rotation_samples(n_base: int = 1000, symmetrise: bool = True) -> np.ndarray:
    """Equal-weight SO(3) quadrature nodes as unit quaternions (w, x, y, z).

    ``n_base`` super-Fibonacci points, each left-multiplied by the 24 octahedral
    rotations when ``symmetrise`` (24*n_base nodes).  The symmetrised set is
    closed under left multiplication by the cube group, which makes the tensor
    template exactly equivariant under the 24 grid-preserving rotations.
    """
    base = super_fibonacci(n_base)
    if not symmetrise:
        return base
    g = octahedral_quaternions()
    q = _qmul(g[:, None, :], base[None, :, :]).reshape(-1, 4)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


# --------------------------------------------------------------------------
# templates: sums of anisotropic Gaussian blobs
# --------------------------------------------------------------------------


@dataclass
class BlobTemplate:
    L: int                      # box edge (voxels)
    centres: np.ndarray         # (B, 3) blob centres relative to the box centre, (x, y, z)
    axes: np.ndarray            # (B, 3, 3) blob principal axes (columns)
    sigmas: np.ndarray          # (B, 3)
    amplitude: float = 1.0

    @property
    def centre(self) -> int:
        return self.L // 2

    def evaluate(self, pts: np.ndarray) -> np.ndarray:
        """Density at points given relative to the template centre, (..., 3) in (x, y, z)."""
        pts = np.asarray(pts, dtype=np.float64)
        out = np.zeros(pts.shape[:-1])
        for b in range(len(self.centres)):
            d = pts - self.centres[b]
            loc = d @ self.axes[b]               # coordinates along the blob axes
            out += np.exp(-0.5 * np.sum((loc / self.sigmas[b]) ** 2, axis=-1))
        return self.amplitude * out

    def volume(self) -> np.ndarray:
        """L^3 float64 array [z][y][x]; voxel (x, y, z) sits at (x, y, z) - centre."""
        idx = np.arange(self.L, dtype=np.float64) - self.centre
        zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
        return self.evaluate(np.stack([xx, yy, zz], axis=-1))


def blob_template(rng: np.random.Generator, L: int, n_blobs: int,
                  sigma_lo: float = 1.5, sigma_hi: float = 3.0,
                  max_offset: float = 4.0) -> BlobTemplate:
    centres = rng.uniform(-max_offset, max_offset, size=(n_blobs, 3))
    axes = random_rotations(rng, n_blobs)
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=(n_blobs, 3))
    return BlobTemplate(L=L, centres=centres, axes=axes, sigmas=sigmas)


# --------------------------------------------------------------------------
# tomograms
# --------------------------------------------------------------------------


def place_centres(rng: np.random.Generator, shape, n: int, min_sep: float,
                  margin: int, max_tries: int = 2000) -> np.ndarray:
    """Integer (z, y, x) centres in [margin, dim-1-margin], pairwise >= min_sep apart.

    Rejection sampling on a hashed grid; stops early (fewer than n) if the
    volume is full.
    """
    nz, ny, nx = shape
    lo = np.array([margin] * 3)
    hi = np.array([nz - 1 - margin, ny - 1 - margin, nx - 1 - margin])
    if np.any(hi < lo):
        return np.zeros((0, 3), dtype=np.int64)
    cell = max(min_sep, 1.0)
    grid: dict = {}
    out = []
    tries = 0
    while len(out) < n and tries < max_tries * max(n, 1):
        tries += 1
        p = rng.integers(lo, hi + 1)
        key = tuple((p // cell).astype(int))
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    for q in grid.get((key[0] + dz, key[1] + dy, key[2] + dx), ()):
                        if np.sum((p - q) ** 2) < min_sep * min_sep:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out.append(p)
            grid.setdefault(key, []).append(p)
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def render_copies(shape, tmpl: BlobTemplate, centres: np.ndarray, rots: np.ndarray,
                  scale: float = 1.0, dtype=np.float32) -> np.ndarray:
    """Analytic rendering: copy j contributes tmpl(R_j^T (p - x_j)) at voxel p."""
    vol = np.zeros(shape, dtype=dtype)
    half = tmpl.L // 2 + 2
    nz, ny, nx = shape
    for j in range(len(centres)):
        cz, cy, cx = (int(v) for v in centres[j])
        z0, z1 = max(cz - half, 0), min(cz + half + 1, nz)
        y0, y1 = max(cy - half, 0), min(cy + half + 1, ny)
        x0, x1 = max(cx - half, 0), min(cx + half + 1, nx)
        zz, yy, xx = np.meshgrid(np.arange(z0, z1) - cz, np.arange(y0, y1) - cy,
                                 np.arange(x0, x1) - cx, indexing="ij")
        d = np.stack([xx, yy, zz], axis=-1).astype(np.float64)
        loc = d @ rots[j]                     # row vector times R == R^T d
        vol[z0:z1, y0:y1, x0:x1] += (scale * tmpl.evaluate(loc)).astype(dtype)
    return vol


def missing_wedge(vol: np.ndarray, half_angle_deg: float = 60.0, workers: int = -1) -> np.ndarray:
    """Zero Fourier coefficients with |k_z| > tan(angle) |k_x| (tilt axis y, beam z); DC kept."""
    import scipy.fft as sfft
    spec = sfft.rfftn(vol, workers=workers)
    nz, ny, nx = vol.shape
    kz = np.fft.fftfreq(nz)[:, None, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    t = math.tan(math.radians(half_angle_deg))
    drop = np.abs(kz) > t * np.abs(kx)        # (nz, 1, nx//2+1); the DC bin is never dropped
    spec *= ~drop
    return sfft.irfftn(spec, s=vol.shape, workers=workers).astype(vol.dtype)


def ball(L: int, r: float) -> np.ndarray:
    idx = np.arange(L) - L // 2
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    return (xx * xx + yy * yy + zz * zz) <= r * r


@dataclass
class Workload:
    name: str
    volume: np.ndarray                 # float32 [z][y][x]
    template: np.ndarray               # float32 L^3
    template_model: BlobTemplate
    mask_radius: float
    degree: int
    centres: np.ndarray                # (N, 3) planted centres (z, y, x)
    rotations: np.ndarray              # (N, 3, 3) planted rotations
    params: dict = field(default_factory=dict)
    quaternions: np.ndarray | None = None   # (N, 4) planted rotations (w, x, y, z), w >= 0


def start_vectors(seed: int = 16, count: int = 16, dim: int = 3) -> np.ndarray:
    """Fixed start vectors of the multi-start search: Gaussian, normalised, upper hemisphere.

    Returned as float32 (both sides consume exactly these values).
    """
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, dim))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v[v[:, -1] < 0] *= -1.0
    return v.astype(np.float32)


def make_tomogram(name: str, shape, L: int, n_blobs: int, n_copies: int, min_sep: float,
                  mask_radius: float, degree: int, seed: int, snr: float | None,
                  wedge: bool, copy_amplitude: float | None = None,
                  template_seed: int | None = None) -> Workload:
    """Tomogram of Gaussian noise plus analytically rendered rotated template copies.

    ``snr=None`` means unit-variance noise with copies scaled to peak
    ``copy_amplitude``; otherwise the noise variance is the template variance
    over its mask divided by ``snr``.
    """
    rng = np.random.default_rng(seed)
    trng = np.random.default_rng(seed if template_seed is None else template_seed)
    tmpl = blob_template(trng, L, n_blobs)
    tvol = tmpl.volume()
    centres = place_centres(rng, shape, n_copies, min_sep, margin=L // 2 + 1)
    rots = random_rotations(rng, len(centres))
    if snr is None:
        amp = copy_amplitude if copy_amplitude is not None else 0.5
        scale = amp / float(tvol.max())
        sig = render_copies(shape, tmpl, centres, rots, scale=scale)
        noise_sd = 1.0
    else:
        scale = 1.0
        sig = render_copies(shape, tmpl, centres, rots, scale=scale)
        m = ball(L, mask_radius)
        noise_sd = math.sqrt(float(np.var(tvol[m])) / snr)
    vol = sig
    vol += (noise_sd * rng.standard_normal(shape, dtype=np.float32)).astype(np.float32)
    if wedge:
        vol = missing_wedge(vol)
    return Workload(name=name, volume=np.ascontiguousarray(vol, dtype=np.float32),
                    template=(scale * tvol).astype(np.float32), template_model=tmpl,
                    mask_radius=mask_radius, degree=degree, centres=centres, rotations=rots,
                    params=dict(shape=tuple(shape), L=L, n_blobs=n_blobs, n_copies=n_copies,
                                min_sep=min_sep, seed=seed, snr=snr, wedge=wedge,
                                noise_sd=noise_sd))


def grid_tomogram(name: str, grid: int, spacing: int, L: int, n_blobs: int, mask_radius: float,
                  degree: int, seed: int, snr: float, template_seed: int,
                  margin: int | None = None, wedge: bool = False) -> Workload:
    """A grid x grid x grid lattice of rotated template copies in Gaussian noise,
    as in the paper's synthetic tomograms (Sec. 4.1: a 5 x 5 x 5 grid of 125
    randomly rotated copies; noise at a stated SNR).  Copy rotations are
    Haar-uniform quaternions, kept in ``quaternions``; the noise variance is the
    template's variance over its mask divided by ``snr``.  With ``wedge`` the
    tomogram (signal and noise) loses the +-60 degree missing wedge; the
    template is returned unfiltered (the wedge lies in the tomogram's frame, so
    filtering the template before it is rotated would turn the wedge with it)."""
    rng = np.random.default_rng(seed)
    tmpl = blob_template(np.random.default_rng(template_seed), L, n_blobs)
    tvol = tmpl.volume()
    m0 = L // 2 + 2 if margin is None else margin
    edge = 2 * m0 + (grid - 1) * spacing + 1
    shape = (edge, edge, edge)
    ax = m0 + spacing * np.arange(grid)
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    centres = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], 1).astype(np.int64)
    quats = random_quaternions(rng, len(centres))
    rots = _quat_to_rot(quats)
    sig = render_copies(shape, tmpl, centres, rots)
    noise_sd = math.sqrt(float(np.var(tvol[ball(L, mask_radius)])) / snr)
    vol = sig + (noise_sd * rng.standard_normal(shape, dtype=np.float32)).astype(np.float32)
    if wedge:
        vol = missing_wedge(vol)
    return Workload(name=name, volume=np.ascontiguousarray(vol, dtype=np.float32),
                    template=tvol.astype(np.float32), template_model=tmpl,
                    mask_radius=mask_radius, degree=degree, centres=centres, rotations=rots,
                    params=dict(shape=shape, L=L, n_blobs=n_blobs, grid=grid, spacing=spacing,
                                seed=seed, snr=snr, noise_sd=noise_sd, template_seed=template_seed,
                                wedge=wedge),
                    quaternions=quats)


# Workload recipes.  The names carry the sizes; "r" is the mask radius.
CONFIGS = {
    "c1_64cube_n4": dict(shape=(64, 64, 64), L=16, n_blobs=3, n_copies=5, min_sep=16,
                         mask_radius=7.0, degree=4, seed=1, snr=None, wedge=False,
                         copy_amplitude=0.5),
    "c2_256cube_n6": dict(shape=(256, 256, 256), L=32, n_blobs=4, n_copies=200, min_sep=32,
                          mask_radius=14.0, degree=6, seed=2, snr=0.1, wedge=True),
    "c3_512x928x928_n6": dict(shape=(512, 928, 928), L=40, n_blobs=5, n_copies=2000,
                              min_sep=40, mask_radius=17.0, degree=6, seed=3, snr=0.05,
                              wedge=True),
}


def make_config(name: str, **overrides) -> Workload:
    p = dict(CONFIGS[name])
    p.update(overrides)
    return make_tomogram(name, **p)


def batch_items(seed: int = 5, n_items: int = 64, edges=(96, 128, 160, 192),
                template_edges=(24, 32, 40), radii=(10.0, 14.0, 17.0),
                copies=(20, 60), snr: float = 0.1):
    """Uneven subtomogram batch: each item holds copies of one of several templates."""
    rng = np.random.default_rng(seed)
    templates = []
    for i, (L, r) in enumerate(zip(template_edges, radii)):
        trng = np.random.default_rng(seed * 1000 + i)
        tm = blob_template(trng, L, 4)
        templates.append((tm, r))
    items = []
    for k in range(n_items):
        e = int(rng.choice(edges))
        ti = int(rng.integers(len(templates)))
        tm, r = templates[ti]
        n = int(rng.integers(copies[0], copies[1] + 1))
        centres = place_centres(rng, (e, e, e), n, r, margin=tm.L // 2 + 1)
        rots = random_rotations(rng, len(centres))
        sig = render_copies((e, e, e), tm, centres, rots)
        m = ball(tm.L, r)
        sd = math.sqrt(float(np.var(tm.volume()[m])) / snr)
        vol = sig + (sd * rng.standard_normal((e, e, e), dtype=np.float32)).astype(np.float32)
        items.append(dict(volume=np.ascontiguousarray(vol, dtype=np.float32), template=ti,
                          centres=centres, rotations=rots))
    return [(tm.volume().astype(np.float32), r, tm) for tm, r in templates], items
