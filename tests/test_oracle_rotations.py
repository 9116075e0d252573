"""Pins of the oracle's rotation helpers and of the rotation sample sets."""
import math

import numpy as np
import pytest

import synth
from oracle import rotations as rot
from oracle import sym


def test_quaternion_matches_rodrigues():
    rng = np.random.default_rng(0)
    for _ in range(20):
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        ang = rng.uniform(-np.pi, np.pi)
        q = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis])
        assert np.allclose(rot.quat_to_matrix(q), rot.axis_angle_matrix(axis, ang), atol=1e-13)


def test_quaternion_product_composes():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a, b = rng.standard_normal(4), rng.standard_normal(4)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        assert np.allclose(rot.quat_to_matrix(rot.quat_mul(a, b)),
                           rot.quat_to_matrix(a) @ rot.quat_to_matrix(b), atol=1e-13)


def test_cube_group():
    G = rot.cube_group()
    assert len(G) == 24
    keys = {tuple(np.round(g).astype(int).ravel()) for g in G}
    for a in G:
        for b in G:
            assert tuple(np.round(a @ b).astype(int).ravel()) in keys


def test_synth_octahedral_quaternions_are_cube_group():
    keys = {tuple(np.round(g).astype(int).ravel()) for g in rot.cube_group()}
    got = {tuple(np.round(rot.quat_to_matrix(q)).astype(int).ravel())
           for q in synth.octahedral_quaternions()}
    assert got == keys
    for q in synth.octahedral_quaternions():
        R = rot.quat_to_matrix(q)
        assert np.allclose(R, np.round(R), atol=1e-14)


def test_trilinear_exact_on_affine():
    L = 9
    p = rot.box_points(L)
    f = 0.3 + 1.5 * p[..., 0] - 0.7 * p[..., 1] + 2.0 * p[..., 2]
    rng = np.random.default_rng(2)
    pts = rng.uniform(0, L - 1, size=(200, 3))
    want = 0.3 + 1.5 * pts[:, 0] - 0.7 * pts[:, 1] + 2.0 * pts[:, 2]
    assert np.allclose(rot.trilinear_sample(f, pts), want, atol=1e-12)
    # outside the box every corner is dropped
    assert np.all(rot.trilinear_sample(f, np.array([[-1.5, 3, 3], [3, 3, L + 0.5]])) == 0)


def test_cube_rotation_is_voxel_permutation():
    rng = np.random.default_rng(3)
    L = 11                                      # odd: the box is symmetric about c
    t = rng.standard_normal((L, L, L))
    c = L // 2
    idx = np.arange(L) - c
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    P = np.stack([xx, yy, zz], axis=-1)
    for G in rot.cube_group():
        tr = rot.rotate_template(t, G)
        src = np.rint(P @ G).astype(int) + c     # G^T p
        want = t[src[..., 2], src[..., 1], src[..., 0]]
        assert np.allclose(tr, want, atol=1e-12)


def test_rotation_samples_unit_and_closed():
    q = synth.rotation_samples(10)
    assert q.shape == (240, 4)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0)
    # closed under left multiplication by the cube group (up to sign)
    key = lambda v: tuple(np.round(v * np.sign(v[np.argmax(np.abs(v))]), 9))
    keys = {key(v) for v in q}
    for g in synth.octahedral_quaternions()[:6]:
        for v in q[:30]:
            assert key(rot.quat_mul(g, v)) in keys


@pytest.mark.parametrize("n", [2, 4, 6])
def test_rotation_sample_moments_s2(n):
    # equal-weight SO(3) nodes: the images v = R a are uniform on S^2, so their
    # monomial means approach the sphere moments (Sec. 3.4: uniform sampling)
    q = synth.rotation_samples(1000)
    v = np.stack([rot.quat_to_matrix(x)[:, 2] for x in q])
    means = sym.monomials(v, n).mean(axis=0)
    want = np.array([sym.sphere_moment(a) for a in sym.multi_indices(n, 3)])
    assert np.max(np.abs(means - want)) < 2e-3


@pytest.mark.parametrize("n", [2, 4])
def test_rotation_sample_moments_s3(n):
    q = synth.rotation_samples(1000, symmetrise=False)
    means = sym.monomials(q, n).mean(axis=0)
    want = np.array([sym.sphere_moment(a) for a in sym.multi_indices(n, 4)])
    assert np.max(np.abs(means - want)) < 2e-3


def test_random_rotations_are_rotations():
    R = synth.random_rotations(np.random.default_rng(4), 50)
    for r in R:
        assert np.allclose(r @ r.T, np.eye(3), atol=1e-12)
        assert np.isclose(np.linalg.det(r), 1.0)
