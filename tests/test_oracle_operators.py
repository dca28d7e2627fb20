"""Pins of the oracle's operators E, E^H, A = E^H E + lambda I (CPU only).

* adjoint identity <E x, y> = <x, E^H y> (invariant) at 2D/3D shapes,
  shared and per-batch maps;
* the paper's Eq. (1) (Section "Sensitivity-weighted multicoil image
  reconstruction"): with full sampling, E^H y times nvox^(-1/2) equals
  sum_i conj(S_i) F^{-1}(Y_i) with F^{-1} the centred inverse DFT scaled by
  1/nvox, evaluated here by brute-force double sums;
* full sampling with sum_c |S_c|^2 = 1 gives E^H E = I (special case);
* the readout-decoupled (hybrid) form of E^H E, built here from numpy 1D
  FFTs along y only, equals the composed oracle A (identity);
* the dense projector F_c^H diag(M) F_c is Hermitian, idempotent and
  circulant (brute force, N <= 64);
* mask semantics: E writes exact zeros off the mask; E^H ignores y there.
"""
import numpy as np
import pytest

import oracle
from paper_1807_11830_amd import synth


def _cn(shape, seed):
    return synth.complex_normal(shape, seed)


def _vdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


CASES_2D = [  # (ny, nx, ncoils, batch, per_batch_maps)
    (8, 8, 2, 1, False),
    (12, 16, 3, 2, True),
    (64, 64, 4, 2, False),
    (10, 6, 2, 1, False),
    (9, 7, 3, 1, False),
]


@pytest.mark.parametrize("ny,nx,nc,b,per", CASES_2D)
def test_adjoint_identity_2d(ny, nx, nc, b, per):
    x = _cn((b, ny, nx), 1)
    y = _cn((b, nc, ny, nx), 2)
    maps = _cn((b, nc, ny, nx) if per else (nc, ny, nx), 3)
    mask = (np.arange(ny) % 3 != 1).astype(np.uint8)
    lhs = _vdot(oracle.E(x, maps, mask), y)
    rhs = _vdot(x, oracle.EH(y, maps, mask))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("nz,ny,nx,nc,b", [(4, 6, 8, 2, 1), (8, 16, 16, 2, 2), (3, 5, 4, 2, 1)])
def test_adjoint_identity_3d(nz, ny, nx, nc, b):
    x = _cn((b, nz, ny, nx), 4)
    y = _cn((b, nc, nz, ny, nx), 5)
    maps = _cn((nc, nz, ny, nx), 6)
    mask = (np.random.default_rng(1).random((nz, ny)) < 0.4).astype(np.uint8)
    lhs = _vdot(oracle.E(x, maps, mask, ndim=3), y)
    rhs = _vdot(x, oracle.EH(y, maps, mask, ndim=3))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _centred_inverse_brute(Y):
    """Centred inverse 2D DFT with 1/(Ny Nx) scale, as explicit double sums:
    out[n] = 1/N sum_k Y[k] exp(+2 pi i (k - h)(n - h) / N) per axis."""
    ny, nx = Y.shape

    def kern(n):
        h = n // 2
        j = np.arange(n) - h
        e = np.outer(j, j) % n
        return np.exp(2j * np.pi * e / n)

    return kern(ny) @ Y @ kern(nx).T / (ny * nx)


def test_eq1_fully_sampled_reconstruction():
    ny, nx, nc = 8, 8, 2
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((1, nc, ny, nx)) + 1j * rng.standard_normal((1, nc, ny, nx))
    S = rng.standard_normal((nc, ny, nx)) + 1j * rng.standard_normal((nc, ny, nx))
    # Eq. (1): M = sum_i S_i^* F^{-1}(Y_i)
    m_eq1 = sum(np.conj(S[i]) * _centred_inverse_brute(Y[0, i]) for i in range(nc))
    full = np.ones(ny, np.uint8)
    got = oracle.EH(Y, S, full)[0] * oracle.eq1_factor(ny * nx)
    assert np.linalg.norm(got - m_eq1) <= 1e-12 * np.linalg.norm(m_eq1)


@pytest.mark.parametrize("n,nc", [(8, 2), (64, 4), (30, 3)])
def test_full_sampling_is_identity(n, nc):
    maps = synth.coil_maps2d(n, nc)
    assert np.allclose(np.sum(np.abs(maps) ** 2, axis=0), 1.0, atol=1e-15)
    x = _cn((1, n, n), 8)
    q = oracle.A(x, maps, np.ones(n, np.uint8))
    assert np.linalg.norm(q - x) <= 1e-12 * np.linalg.norm(x)


def _hybrid_normal(p, maps, mask):
    """q = sum_c conj(S_c) ifft_y( M_u fft_y(S_c p) ), M_u[k] = M[(k + ny/2) % ny]:
    the centred 2D E^H E with a per-line mask reduces to 1D transforms along y
    with an uncentred mask (the readout transforms cancel)."""
    ny = p.shape[-2]
    mu = mask[(np.arange(ny) + ny // 2) % ny].astype(float)[:, None]
    q = np.zeros_like(p)
    for c in range(maps.shape[0]):
        u = maps[c] * p
        q += np.conj(maps[c]) * np.fft.ifft(mu * np.fft.fft(u, axis=0), axis=0)
    return q


@pytest.mark.parametrize("n,nc,accel", [(64, 4, 2.0), (128, 8, 4.0), (32, 3, 3.0)])
def test_hybrid_identity(n, nc, accel):
    maps = synth.coil_maps2d(n, nc)
    mask = synth.mask_variable_density(n, accel, 8)
    p = _cn((1, n, n), 12)
    q_comp = oracle.A(p, maps, mask)[0]
    q_hyb = _hybrid_normal(p[0], maps, mask)
    assert np.linalg.norm(q_comp - q_hyb) <= 1e-13 * np.linalg.norm(q_comp)


@pytest.mark.parametrize("n", [8, 16, 64])
def test_dense_projector_properties(n):
    mask = synth.mask_variable_density(n, 2.0, 2, seed=3)
    eye = np.eye(n, dtype=complex)
    F = np.stack([oracle.centred1d(eye[:, j], -1) for j in range(n)], axis=1)
    P = F.conj().T @ np.diag(mask.astype(float)) @ F
    assert np.allclose(F.conj().T @ F, eye, atol=1e-13)
    assert np.allclose(P, P.conj().T, atol=1e-13)
    assert np.allclose(P @ P, P, atol=1e-13)
    for i in range(n):
        assert np.allclose(np.roll(P[0], i), P[i], atol=1e-13)
    assert abs(np.trace(P).real - mask.sum()) <= 1e-12


def test_mask_semantics():
    n, nc = 16, 2
    maps = _cn((nc, n, n), 20)
    mask = synth.mask_regular(n, 2, 4)
    x = _cn((1, n, n), 21)
    y = oracle.E(x, maps, mask)
    assert np.all(y[:, :, mask == 0, :] == 0)
    assert np.all(np.abs(y[:, :, mask == 1, :]) > 0)
    y2 = _cn((1, nc, n, n), 22)
    y3 = y2.copy()
    y3[:, :, mask == 0, :] = 1e3 * _cn(y3[:, :, mask == 0, :].shape, 23)
    assert np.array_equal(oracle.EH(y2, maps, mask), oracle.EH(y3, maps, mask))


def test_lambda_and_batch_independence():
    n, nc = 16, 3
    maps = _cn((2, nc, n, n), 30)
    mask = synth.mask_regular(n, 2, 4)
    p = _cn((2, n, n), 31)
    q0 = oracle.A(p, maps, mask)
    q1 = oracle.A(p, maps, mask, lam=0.25)
    assert np.allclose(q1 - q0, 0.25 * p, atol=1e-13)
    for b in range(2):
        qb = oracle.A(p[b:b + 1], maps[b], mask)
        assert np.array_equal(qb[0], q0[b])
    # shared maps equal per-batch copies
    qs = oracle.A(p, maps[0], mask)
    qc = oracle.A(p, np.stack([maps[0], maps[0]]), mask)
    assert np.array_equal(qs, qc)


def test_rss_matches_library_definition():
    n, nc = 16, 3
    y = _cn((2, nc, n, n), 40)
    got = oracle.rss(y)
    imgs = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(y, axes=(-2, -1)), norm="ortho"), axes=(-2, -1))
    ref = np.sqrt(np.sum(np.abs(imgs) ** 2, axis=1))
    assert np.allclose(got, ref, atol=1e-13)
