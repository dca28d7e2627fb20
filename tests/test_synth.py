"""Synthetic input generators: determinism, normalisation, mask counts."""
import json
import os

import numpy as np
import pytest

from paper_1807_11830_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "synth_hashes.json")


def test_maps_normalised():
    for n, c in ((64, 4), (256, 12), (30, 3)):
        m = synth.coil_maps2d(n, c)
        assert m.shape == (c, n, n)
        assert np.allclose(np.sum(np.abs(m) ** 2, axis=0), 1.0, atol=1e-14)
    m3 = synth.coil_maps3d(16, 16, 8, 4)
    assert np.allclose(np.sum(np.abs(m3) ** 2, axis=0), 1.0, atol=1e-14)


def test_phantom_ranges():
    p = synth.phantom2d(64, seed=11)
    assert p.dtype == np.complex128 and np.all(p.imag == 0)
    assert p.real.min() >= 0 and p.real.max() > 0.1
    assert np.count_nonzero(p) > 64 * 64 // 20
    v = synth.phantom3d(32, 32, 16)
    assert v.shape == (16, 32, 32) and v.real.max() > 0.1


def test_mask_counts():
    m = synth.mask_regular(64, 2, 8)
    assert m.sum() == 36 and all(m[28:36]) and m[1] == 0
    for n, r in ((256, 4), (384, 4), (128, 2), (192, 3), (320, 4)):
        mv = synth.mask_variable_density(n, r, 24)
        assert mv.sum() == round(n / r)
        assert all(mv[n // 2 - 12: n // 2 + 12])
    m2 = synth.mask_variable_density_2d(256, 128, 6, (32, 32))
    assert m2.shape == (128, 256) and m2.sum() == round(256 * 128 / 6)
    assert m2[64 - 16: 64 + 16, 128 - 16: 128 + 16].all()


def test_generators_deterministic():
    with open(GOLDEN) as f:
        ref = json.load(f)
    got = {
        "phantom2d_64_s11": synth.sha256(synth.phantom2d(64, seed=11)),
        "maps2d_64_c4": synth.sha256(synth.coil_maps2d(64, 4)),
        "mask_regular_64": synth.sha256(synth.mask_regular(64, 2, 8)),
        "mask_vd_256_r4": synth.sha256(synth.mask_variable_density(256, 4.0, 24)),
        "noise_4x64x64": synth.sha256(synth.complex_noise((4, 64, 64))),
    }
    # every input is pinned, the float arrays included: numpy's generators
    # (PCG64, ziggurat normals) are platform independent, and the phantom and
    # maps use only basic arithmetic, exp, sin and cos of the same numpy
    # build on every machine that runs this suite
    assert set(got) == set(ref)
    for k, v in got.items():
        assert v == ref[k], k


def test_request_stream():
    reqs = synth.request_stream(32, rate=100.0)
    assert len(reqs) == 32
    assert all(r["n"] in (128, 192, 256, 320) and r["ncoils"] in (8, 16, 32) and r["accel"] in (2, 3, 4) for r in reqs)
    t = [r["arrival"] for r in reqs]
    assert t == sorted(t)
    assert reqs == synth.request_stream(32, rate=100.0)
