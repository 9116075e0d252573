"""Constants the paper fixes, and properties of the synthetic input generator."""
import json
import math
import os

import numpy as np

import synth
from oracle import sym, ttm

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_paper_constants():
    g = json.load(open(GOLD))
    a = g["filter_a"]["value"]
    assert np.allclose(ttm.filter_taps(a), [0.2, 0.6, 0.2])
    assert 1 - 4 * a == g["filter_min_response"]["value"] or math.isclose(1 - 4 * a, 0.2)
    assert sym.n_components(4, 4) == g["components_n4_d4"]["value"]


def test_generator_is_seeded_and_shaped():
    a = synth.make_tomogram("x", (24, 26, 28), L=8, n_blobs=3, n_copies=3, min_sep=8,
                            mask_radius=3.0, degree=4, seed=5, snr=0.5, wedge=True)
    b = synth.make_tomogram("x", (24, 26, 28), L=8, n_blobs=3, n_copies=3, min_sep=8,
                            mask_radius=3.0, degree=4, seed=5, snr=0.5, wedge=True)
    assert a.volume.dtype == np.float32 and a.volume.shape == (24, 26, 28)
    assert np.array_equal(a.volume, b.volume)
    assert a.template.shape == (8, 8, 8)
    for i in range(len(a.centres)):
        for j in range(i):
            assert np.linalg.norm(a.centres[i] - a.centres[j]) >= 8


def test_missing_wedge_zeroes_the_wedge_and_keeps_dc():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((16, 8, 16)).astype(np.float32) + 3.0
    out = synth.missing_wedge(v)
    spec = np.fft.rfftn(out)
    kz = np.fft.fftfreq(16)[:, None, None]
    kx = np.fft.rfftfreq(16)[None, None, :]
    drop = np.broadcast_to(np.abs(kz) > math.tan(math.radians(60)) * np.abs(kx), spec.shape)
    assert np.abs(spec[drop]).max() < 1e-3
    assert np.isclose(out.mean(), v.mean(), atol=1e-5)


def test_start_vectors_upper_hemisphere():
    s = synth.start_vectors()
    assert s.shape == (16, 3) and s.dtype == np.float32
    assert np.allclose(np.linalg.norm(s.astype(np.float64), axis=1), 1, atol=1e-6)
    assert np.all(s[:, 2] >= 0)
