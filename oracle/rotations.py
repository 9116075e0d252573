"""Rotations (FP64).  TEST INFRASTRUCTURE ONLY (see oracle/__init__).

* Unit quaternions q = (w, x, y, z), Hamilton product; R(q) rotates vectors
  (x, y, z).  The paper encodes rotations of SO(3) as unit quaternions with
  d' = 4 (Sec. 3, after Eq. tt).
* The rotated template t'_q (Alg. 1, "rotate t' according to q") is the
  trilinear pull-back t'_q(p) = t'(c + R(q)^T (p - c)), zero outside the box.
  The paper does not state the interpolation; this reading keeps the identity
  between the tensor field and rotation-sampled TM exact (both use the same
  rotated templates).
* The cube group: the 24 signed permutation matrices of determinant +1.  They
  map the voxel grid onto itself about a voxel centre.

Pins: R(q) against the Rodrigues formula and R(q1 q2) = R(q1) R(q2); the cube
group's closure; trilinear sampling of an affine function is exact; rotation
by a cube-group element equals the voxel permutation.
"""
from __future__ import annotations

import itertools

import numpy as np


def quat_to_matrix(q) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def quat_mul(a, b) -> np.ndarray:
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def axis_angle_matrix(axis, angle) -> np.ndarray:
    """Rodrigues: I + sin(a) K + (1 - cos(a)) K^2."""
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def cube_group() -> list:
    """The 24 rotation matrices that permute the axes with signs."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            G = np.zeros((3, 3))
            for i, j in enumerate(perm):
                G[i, j] = signs[i]
            if np.linalg.det(G) > 0:
                out.append(G)
    return out


def trilinear_sample(vol: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Sample vol ([z][y][x]) at continuous (x, y, z) points; zero outside the box.

    Each of the 8 cell corners contributes its value times its trilinear
    weight when it lies inside the array, nothing otherwise.
    """
    nz, ny, nx = vol.shape
    pts = np.asarray(pts, dtype=np.float64)
    i0 = np.floor(pts).astype(np.int64)
    fr = pts - i0
    out = np.zeros(pts.shape[:-1])
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                ix, iy, iz = i0[..., 0] + dx, i0[..., 1] + dy, i0[..., 2] + dz
                wgt = ((fr[..., 0] if dx else 1 - fr[..., 0]) *
                       (fr[..., 1] if dy else 1 - fr[..., 1]) *
                       (fr[..., 2] if dz else 1 - fr[..., 2]))
                inside = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny) & (iz >= 0) & (iz < nz)
                val = np.zeros(pts.shape[:-1])
                val[inside] = vol[iz[inside], iy[inside], ix[inside]]
                out += wgt * val
    return out


def box_points(L: int) -> np.ndarray:
    """Voxel coordinates (x, y, z) of an L^3 box, shape (L, L, L, 3) indexed [z][y][x]."""
    idx = np.arange(L, dtype=np.float64)
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.stack([xx, yy, zz], axis=-1)


def rotate_template(t: np.ndarray, R: np.ndarray) -> np.ndarray:
    """t_R(p) = t(c + R^T (p - c)) with c = L//2 on every axis (cubic box)."""
    L = t.shape[0]
    c = float(L // 2)
    p = box_points(L) - c
    src = p @ R + c                  # row vector p times R == R^T p
    return trilinear_sample(t, src)
