"""Pins of the oracle's transforms (CPU only).

The oracle's FFT is checked against the defining O(N^2) sum evaluated here
with numpy (brute force), against numpy.fft (an independent library
routine), and against closed forms: Parseval, the inverse, impulse
responses of the centred transform, and the checkerboard form of centring.
"""
import numpy as np
import pytest

import oracle

LENGTHS = list(range(1, 17)) + [18, 20, 24, 25, 27, 30, 45, 49, 64, 128, 160, 192, 256, 320, 384]


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _brute_dft(v, sign):
    n = v.size
    k = np.arange(n)
    # exponent reduced mod n in integers before the float conversion
    e = np.outer(k, k) % n
    return np.exp(sign * 2j * np.pi * e / n) @ v


@pytest.mark.parametrize("n", LENGTHS)
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_brute_force(n, sign):
    v = _rand(n, n)
    ref = _brute_dft(v, sign)
    got = oracle.fft1d(v, sign)
    assert np.linalg.norm(got - ref) <= 1e-13 * max(1.0, np.linalg.norm(ref))
    got_direct = oracle.dft1d_direct(v, sign)
    assert np.linalg.norm(got_direct - ref) <= 1e-13 * max(1.0, np.linalg.norm(ref))


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_numpy(n):
    v = _rand(n, 100 + n)
    assert np.allclose(oracle.fft1d(v, -1), np.fft.fft(v), rtol=0, atol=1e-12 * np.sqrt(n))
    assert np.allclose(oracle.fft1d(v, +1), n * np.fft.ifft(v), rtol=0, atol=1e-12 * np.sqrt(n))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 15, 16, 64, 160, 192, 256, 320, 384])
def test_centred_unitary_and_inverse(n):
    v = _rand(n, 7 * n)
    f = oracle.centred1d(v, -1)
    assert abs(np.linalg.norm(f) - np.linalg.norm(v)) <= 1e-14 * np.linalg.norm(v) * max(1, np.log2(n))
    back = oracle.centred1d(f, +1)
    assert np.linalg.norm(back - v) <= 1e-14 * np.linalg.norm(v) * max(1, np.log2(n))


@pytest.mark.parametrize("n", [8, 9, 10, 16, 64, 160, 256, 384])
def test_centred_matches_numpy_shift_convention(n):
    v = _rand(n, 3 * n)
    ref = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(v))) / np.sqrt(n)
    assert np.allclose(oracle.centred1d(v, -1), ref, atol=1e-13)
    refi = np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(v))) * np.sqrt(n)
    assert np.allclose(oracle.centred1d(v, +1), refi, atol=1e-13)


@pytest.mark.parametrize("n", [8, 10, 16, 64, 160, 256])
def test_centred_impulses(n):
    # An impulse at the centre index n/2 maps to the constant n^(-1/2);
    # an impulse at n/2 + m maps to n^(-1/2) exp(-2 pi i (k - n/2) m / n).
    k = np.arange(n)
    for m in (0, 1, 3, -2):
        v = np.zeros(n, complex)
        v[(n // 2 + m) % n] = 1.0
        expect = np.exp(-2j * np.pi * (k - n // 2) * m / n) / np.sqrt(n)
        assert np.allclose(oracle.centred1d(v, -1), expect, atol=1e-14)
        assert np.allclose(oracle.centred1d(v, +1), np.conj(expect), atol=1e-14)


@pytest.mark.parametrize("n", [8, 12, 16, 64, 256, 10, 14, 30, 160])
def test_checkerboard_form(n):
    # For even n: F_c v = (-1)^(n/2) (-1)^k DFT((-1)^j v) / sqrt(n).
    v = _rand(n, 11 * n)
    s = (-1.0) ** np.arange(n)
    ref = ((-1.0) ** (n // 2)) * s * np.fft.fft(s * v) / np.sqrt(n)
    assert np.allclose(oracle.centred1d(v, -1), ref, atol=1e-13)


def test_centred_nd_is_axis_by_axis():
    rng = np.random.default_rng(5)
    img = rng.standard_normal((6, 8, 10)) + 1j * rng.standard_normal((6, 8, 10))
    ref = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(img), norm="ortho"))
    assert np.allclose(oracle.centred_nd(img, -1), ref, atol=1e-13)
    ref2 = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img[0]), norm="ortho"))
    assert np.allclose(oracle.centred_nd(img[0], -1), ref2, atol=1e-13)
    back = oracle.centred_nd(oracle.centred_nd(img, -1), +1)
    assert np.allclose(back, img, atol=1e-13)
