"""Pins of the oracle's CG-SENSE (CPU only).

* on a tiny problem (8x8, 2 coils, R=2; dimension 64) the k-th CG iterate
  equals the minimiser of the A-norm error over the Krylov space K_k(A, b),
  computed here from a fully re-orthogonalised Arnoldi basis and the dense
  matrix of A (brute force);
* after 64 iterations it equals the least-squares solution of the dense
  system (numpy.linalg.lstsq, a library routine); the A-norm error
  decreases monotonically;
* with Tikhonov lambda the same two checks hold for A + lambda I (dense
  numpy.linalg.solve), and the Krylov check holds for a tiny volume (3D);
* full sampling with sum |S|^2 = 1 and noise-free data recovers the image in
  one iteration (alpha = 1) — a special case;
* stop statuses: zero data -> EXACT at 0, tolerance -> CONVERGED,
  A = 0 (lambda = -1 at full sampling) -> BREAKDOWN, NaN -> NONFINITE;
* batch elements are independent problems;
* the complex64-storage mode (vec32): its iterates are binary32 values, its
  first iterate differs from the fp64 one by a few binary32 roundings only,
  and it recovers the image under full sampling to binary32 precision.
"""
import numpy as np
import pytest

import oracle
from paper_1807_11830_amd import synth


def _tiny():
    n, nc = 8, 2
    # generic (random) sensitivities: the Gaussian-bump maps at 8x8 with two
    # coils make b an eigenvector of A, which ends CG after one step
    maps = 0.5 * synth.complex_normal((nc, n, n), 70)
    mask = synth.mask_regular(n, 2, 2)
    x_true = synth.phantom2d(n, seed=3)[None]
    y = oracle.E(x_true, maps, mask) + synth.complex_noise((1, nc, n, n), 1e-2, 4) * mask[None, None, :, None]
    return n, maps, mask, y


def _dense_A(n, maps, mask):
    dim = n * n
    Ad = np.empty((dim, dim), complex)
    for j in range(dim):
        e = np.zeros(dim, complex)
        e[j] = 1.0
        Ad[:, j] = oracle.A(e.reshape(1, n, n), maps, mask).ravel()
    return Ad


def _krylov_minimiser(Ad, b, k):
    """argmin_{x in K_k(A, b)} ||x - x*||_A = V (V^H A V)^{-1} V^H b."""
    V = np.zeros((b.size, k), complex)
    v = b / np.linalg.norm(b)
    for j in range(k):
        for _ in range(2):  # full re-orthogonalisation, twice
            v = v - V[:, :j] @ (V[:, :j].conj().T @ v)
        v = v / np.linalg.norm(v)
        V[:, j] = v
        v = Ad @ v
    H = V.conj().T @ Ad @ V
    return V @ np.linalg.solve(H, V.conj().T @ b)


def test_cg_iterates_are_krylov_minimisers():
    n, maps, mask, y = _tiny()
    Ad = _dense_A(n, maps, mask)
    assert np.allclose(Ad, Ad.conj().T, atol=1e-13)
    b = oracle.EH(y, maps, mask).ravel()
    for k in (1, 2, 3, 5, 8, 12):
        x, iters, status, _ = oracle.cg(y, maps, mask, k)
        assert iters[0] == k and status[0] == oracle.MAXITER
        ref = _krylov_minimiser(Ad, b, k)
        assert np.linalg.norm(x.ravel() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_cg_converges_to_lstsq_and_error_monotone():
    n, maps, mask, y = _tiny()
    Ad = _dense_A(n, maps, mask)
    b = oracle.EH(y, maps, mask).ravel()
    xs = np.linalg.lstsq(Ad, b, rcond=None)[0]
    errs = []
    for k in range(1, 25):
        x, iters, status, _ = oracle.cg(y, maps, mask, k)
        d = x.ravel() - xs
        errs.append(np.sqrt(max(np.vdot(d, Ad @ d).real, 0.0)))
    assert all(e2 <= e1 * (1 + 1e-9) + 1e-13 for e1, e2 in zip(errs, errs[1:]))
    x, iters, status, _ = oracle.cg(y, maps, mask, 64)
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)


def test_cg_with_lambda_solves_the_regularised_system():
    """With Tikhonov lambda the iterates minimise over the Krylov space of
    A + lambda I, and 64 iterations give the dense solve of
    (A + lambda I) x = E^H y (numpy.linalg.solve): a dropped or mis-signed
    lambda anywhere in the loop fails both."""
    n, maps, mask, y = _tiny()
    lam = 0.3
    Ad = _dense_A(n, maps, mask) + lam * np.eye(n * n)
    b = oracle.EH(y, maps, mask).ravel()
    for k in (2, 5):
        x, _, _, _ = oracle.cg(y, maps, mask, k, lam=lam)
        ref = _krylov_minimiser(Ad, b, k)
        assert np.linalg.norm(x.ravel() - ref) <= 1e-9 * np.linalg.norm(ref)
    x, _, _, _ = oracle.cg(y, maps, mask, 64, lam=lam)
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)
    x0, _, _, _ = oracle.cg(y, maps, mask, 64)
    assert np.linalg.norm(x0.ravel() - xs) > 1e-3 * np.linalg.norm(xs)


def test_cg_3d_iterates_are_krylov_minimisers():
    """The same Krylov pin for a tiny volume (4 x 4 x 4, 2 coils, a random
    (ky, kz) mask; dimension 64): the CG loop at ndim = 3."""
    nz, ny, nx, nc = 4, 4, 4, 2
    maps = 0.5 * synth.complex_normal((nc, nz, ny, nx), 80)
    mask = synth.mask_variable_density_2d(ny, nz, 2.0, (2, 2), seed=81)
    x_true = synth.complex_normal((1, nz, ny, nx), 82)
    y = oracle.E(x_true, maps, mask, ndim=3)
    dim = nx * ny * nz
    Ad = np.empty((dim, dim), complex)
    for j in range(dim):
        e = np.zeros(dim, complex)
        e[j] = 1.0
        Ad[:, j] = oracle.A(e.reshape(1, nz, ny, nx), maps, mask, ndim=3).ravel()
    assert np.allclose(Ad, Ad.conj().T, atol=1e-13)
    b = oracle.EH(y, maps, mask, ndim=3).ravel()
    for k in (1, 3, 6):
        x, iters, status, _ = oracle.cg(y, maps, mask, k, ndim=3)
        assert iters[0] == k and status[0] == oracle.MAXITER
        ref = _krylov_minimiser(Ad, b, k)
        assert np.linalg.norm(x.ravel() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_full_sampling_one_iteration_recovery():
    n, nc = 32, 4
    maps = synth.coil_maps2d(n, nc)
    full = np.ones(n, np.uint8)
    x_true = synth.phantom2d(n, seed=5)[None]
    y = oracle.E(x_true, maps, full)
    x, iters, status, hist = oracle.cg(y, maps, full, 5, tol=1e-10)
    assert status[0] == oracle.CONVERGED and iters[0] == 1
    assert np.linalg.norm(x - x_true) <= 1e-12 * np.linalg.norm(x_true)
    assert hist[0, 1] <= 1e-24 * hist[0, 0]


def test_statuses():
    n, nc = 16, 2
    maps = synth.coil_maps2d(n, nc)
    mask = synth.mask_regular(n, 2, 4)
    zero = np.zeros((1, nc, n, n), complex)
    x, iters, status, hist = oracle.cg(zero, maps, mask, 5)
    assert status[0] == oracle.EXACT and iters[0] == 0 and np.all(x == 0)

    y = oracle.E(synth.phantom2d(n, seed=1)[None], maps, mask)
    x, iters, status, hist = oracle.cg(y, maps, mask, 50, tol=1e-3)
    assert status[0] == oracle.CONVERGED
    k = iters[0]
    assert np.sqrt(hist[0, k] / hist[0, 0]) < 1e-3 <= np.sqrt(hist[0, k - 1] / hist[0, 0])

    full = np.ones(n, np.uint8)
    y = oracle.E(synth.phantom2d(n, seed=1)[None], maps, full)
    x, iters, status, hist = oracle.cg(y, maps, full, 5, lam=-1.0)
    assert status[0] == oracle.BREAKDOWN and iters[0] == 0

    ynan = y.copy()
    ynan[0, 0, 3, 3] = np.nan
    x, iters, status, hist = oracle.cg(ynan, maps, full, 5)
    assert status[0] == oracle.NONFINITE and iters[0] == 0


def test_batch_independence():
    n, nc = 16, 3
    maps = synth.coil_maps2d(n, nc)
    mask = synth.mask_variable_density(n, 2.0, 4)
    xt = np.stack([synth.phantom2d(n, seed=s) for s in (1, 2)])
    y = oracle.E(xt, maps, mask)
    xb, itb, stb, hb = oracle.cg(y, maps, mask, 7)
    for b in range(2):
        x1, it1, st1, h1 = oracle.cg(y[b:b + 1], maps, mask, 7)
        assert np.array_equal(x1[0], xb[b])
        assert np.array_equal(h1[0], hb[b])


@pytest.mark.parametrize("eps", [1e-4])
def test_gradient_finite_differences(eps):
    """grad of L(x) = ||E x - y||^2 is 2 E^H (E x - y) (complex convention
    g = dL/dRe + i dL/dIm): central differences along random directions."""
    n, nc = 8, 2
    maps = synth.complex_normal((nc, n, n), 50) * 0.5
    mask = synth.mask_regular(n, 2, 2)
    x = synth.complex_normal((1, n, n), 51)
    y = synth.complex_normal((1, nc, n, n), 52) * mask[None, None, :, None]

    def L(v):
        r = oracle.E(v, maps, mask) - y
        return np.vdot(r.ravel(), r.ravel()).real

    g = 2.0 * oracle.EH(oracle.E(x, maps, mask) - y, maps, mask)
    for s in range(4):
        d = synth.complex_normal((1, n, n), 60 + s)
        fd = (L(x + eps * d) - L(x - eps * d)) / (2 * eps)
        an = np.vdot(g.ravel(), d.ravel()).real
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_vec32_iterates_are_binary32_and_close_to_fp64():
    n, maps, mask, y = _tiny()
    for k in (1, 6):
        x32, it32, st32, h32 = oracle.cg(y, maps, mask, k, vec32=True)
        x64, it64, st64, h64 = oracle.cg(y, maps, mask, k)
        assert it32[0] == it64[0] == k
        assert np.array_equal(x32, x32.astype(np.complex64).astype(np.complex128))
        d = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
        assert d > 0.0
        # one iteration: x1 = alpha * round32(b), a few roundings of 2^-24
        assert d <= (8 * 2.0 ** -24 if k == 1 else 1e-5)
    assert not np.array_equal(x64, x64.astype(np.complex64).astype(np.complex128))


def test_vec32_full_sampling_recovery():
    n, nc = 32, 4
    maps = synth.coil_maps2d(n, nc)
    full = np.ones(n, np.uint8)
    x_true = synth.phantom2d(n, seed=5)[None]
    y = oracle.E(x_true, maps, full)
    x, iters, status, hist = oracle.cg(y, maps, full, 1, vec32=True)
    assert iters[0] == 1
    assert np.linalg.norm(x - x_true) <= 4 * 2.0 ** -24 * np.linalg.norm(x_true)
