"""Pins of the oracle's 3D operators against an independent construction
(CPU only).

The 3D forward model is y_c = M .* F_c(S_c .* x) with F_c the centred
unitary DFT over all three axes and M the (ky, kz) phase-encode mask,
stored [Nz][Ny] in centred order and broadcast along the readout x (the
multicoil model whose adjoint with M = 1 is the paper's Eq. (1)).  Here E
and E^H are rebuilt from numpy's n-dimensional FFT (pocketfft) with
numpy's own fftshift / ifftshift and an explicit broadcast of the mask, so
that an orientation mistake in how the oracle indexes the [Nz][Ny] mask
(which both E and E^H would share, leaving the adjoint identity intact)
fails this pin.  Sizes use nz != ny and an asymmetric random mask; one odd
axis checks the shift convention for odd lengths too.

A planted mutant (the mask buffer read with the ky and kz strides
swapped) passes the adjoint identity and must fail the fftn pin.
"""
import numpy as np
import pytest

import oracle
from paper_1807_11830_amd import synth


def _fftn_c(v, inverse=False):
    """Centred unitary DFT over the last three axes via numpy.fft."""
    ax = (-3, -2, -1)
    f = np.fft.ifftn if inverse else np.fft.fftn
    return np.fft.fftshift(f(np.fft.ifftshift(v, axes=ax), axes=ax, norm="ortho"), axes=ax)


def _bmask(mask):
    """[Nz][Ny] mask -> broadcast shape [Nz][Ny][1] over the readout x."""
    return mask.astype(float)[:, :, None]


def _E_np(x, maps, mask):
    """x [B][Nz][Ny][Nx], maps [C][Nz][Ny][Nx] -> y [B][C][Nz][Ny][Nx]."""
    return np.stack([np.stack([_fftn_c(maps[c] * x[b]) * _bmask(mask) for c in range(maps.shape[0])])
                     for b in range(x.shape[0])])


def _EH_np(y, maps, mask):
    return np.stack([sum(np.conj(maps[c]) * _fftn_c(y[b, c] * _bmask(mask), inverse=True)
                         for c in range(maps.shape[0])) for b in range(y.shape[0])])


def _case(nz, ny, nx, nc, b, seed):
    rng = np.random.default_rng(seed)
    x = synth.complex_normal((b, nz, ny, nx), seed + 1)
    maps = synth.complex_normal((nc, nz, ny, nx), seed + 2)
    y = synth.complex_normal((b, nc, nz, ny, nx), seed + 3)
    mask = (rng.random((nz, ny)) < 0.45).astype(np.uint8)
    # asymmetric: not equal to its own point reflection or transpose pattern
    mask[0, :] = 0
    mask[:, 1] = 1
    return x, maps, y, mask


SHAPES = [(4, 6, 8, 2, 1), (6, 10, 4, 3, 2), (8, 12, 6, 2, 1), (5, 8, 6, 2, 1), (16, 32, 8, 2, 1)]


@pytest.mark.parametrize("nz,ny,nx,nc,b", SHAPES)
def test_oracle_3d_E_matches_numpy_fftn(nz, ny, nx, nc, b):
    x, maps, y, mask = _case(nz, ny, nx, nc, b, seed=nz * 100 + ny)
    ref = _E_np(x, maps, mask)
    got = oracle.E(x, maps, mask, ndim=3)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("nz,ny,nx,nc,b", SHAPES)
def test_oracle_3d_EH_matches_numpy_fftn(nz, ny, nx, nc, b):
    x, maps, y, mask = _case(nz, ny, nx, nc, b, seed=nz * 100 + ny + 7)
    ref = _EH_np(y, maps, mask)
    got = oracle.EH(y, maps, mask, ndim=3)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_oracle_3d_mask_semantics():
    """E writes exact zeros on every unsampled (kz, ky) line, for every x
    and coil; E^H ignores whatever y holds there."""
    nz, ny, nx, nc = 6, 10, 8, 2
    x, maps, y, mask = _case(nz, ny, nx, nc, 1, seed=5)
    ye = oracle.E(x, maps, mask, ndim=3)
    off = mask == 0
    assert np.all(ye[:, :, off, :] == 0)
    assert np.all(np.abs(ye[:, :, ~off, :]) > 0)
    y2 = y.copy()
    y2[:, :, off, :] = 1e3 * synth.complex_normal(y2[:, :, off, :].shape, 99)
    assert np.array_equal(oracle.EH(y, maps, mask, ndim=3), oracle.EH(y2, maps, mask, ndim=3))


def test_oracle_3d_full_sampling_reduces_to_fftn():
    """With M = 1 and one coil of ones, E is numpy's centred unitary fftn
    and E^H its inverse (library special case)."""
    nz, ny, nx = 4, 6, 10
    x = synth.complex_normal((1, nz, ny, nx), 3)
    ones = np.ones((1, nz, ny, nx), complex)
    full = np.ones((nz, ny), np.uint8)
    assert np.allclose(oracle.E(x, ones, full, ndim=3)[0, 0], _fftn_c(x[0]), atol=1e-13)
    assert np.allclose(oracle.EH(x[:, None], ones, full, ndim=3)[0], _fftn_c(x[0], inverse=True), atol=1e-13)


def _swapped_strides(mask):
    """The planted mistake: the [Nz][Ny] mask buffer read as [Ny][Nz]
    (index y * nz + z instead of z * ny + y), i.e. a transposed reading."""
    nz, ny = mask.shape
    return np.ascontiguousarray(mask.ravel().reshape(ny, nz).T)


def _E_mut(x, maps, mask):
    m = _swapped_strides(mask)
    out = np.empty((x.shape[0], maps.shape[0]) + x.shape[1:], complex)
    for b in range(x.shape[0]):
        for c in range(maps.shape[0]):
            out[b, c] = oracle.centred_nd(maps[c] * x[b], -1) * m[:, :, None]
    return out


def _EH_mut(y, maps, mask):
    m = _swapped_strides(mask)
    out = np.zeros((y.shape[0],) + y.shape[2:], complex)
    for b in range(y.shape[0]):
        for c in range(maps.shape[0]):
            out[b] += np.conj(maps[c]) * oracle.centred_nd(y[b, c] * m[:, :, None], +1)
    return out


def test_transposed_mask_mutant_passes_adjoint_but_fails_fftn_pin():
    nz, ny, nx, nc = 6, 10, 4, 2
    x, maps, y, mask = _case(nz, ny, nx, nc, 1, seed=11)
    assert not np.array_equal(_swapped_strides(mask), mask)
    # the old pin: the adjoint identity cannot see a shared orientation error
    lhs = np.vdot(_E_mut(x, maps, mask).ravel(), y.ravel())
    rhs = np.vdot(x.ravel(), _EH_mut(y, maps, mask).ravel())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the new pin does
    ref = _E_np(x, maps, mask)
    assert np.linalg.norm(_E_mut(x, maps, mask) - ref) > 1e-3 * np.linalg.norm(ref)
    refh = _EH_np(y, maps, mask)
    assert np.linalg.norm(_EH_mut(y, maps, mask) - refh) > 1e-3 * np.linalg.norm(refh)
    # while the unmutated path built from the same primitives passes it
    good = np.stack([np.stack([oracle.centred_nd(maps[c] * x[0], -1) * _bmask(mask) for c in range(nc)])])
    assert np.linalg.norm(good - ref) <= 1e-13 * np.linalg.norm(ref)


def test_oracle_3d_A_matches_numpy_composition():
    """A = E^H E + lambda I in 3D against the fftn construction."""
    nz, ny, nx, nc = 8, 6, 4, 3
    x, maps, y, mask = _case(nz, ny, nx, nc, 1, seed=21)
    ref = _EH_np(_E_np(x, maps, mask), maps, mask) + 0.3 * x
    got = oracle.A(x, maps, mask, lam=0.3, ndim=3)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
