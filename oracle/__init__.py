"""FP64 CPU oracle for multicoil Cartesian SENSE (E, E^H, E^H E, CG, RSS).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never imports, loads or calls it,
and the two share no code.

The arithmetic lives in ``sense_oracle.c`` (plain C99, double complex),
compiled by :func:`build` with gcc into ``libsense_oracle.so`` next to it.
This module only marshals numpy arrays (complex128 / uint8) across ctypes.

Function-by-function citations (the paper is arXiv 1807.11830):

* :func:`EH` with a full mask is the paper's reconstruction equation,
  Section "Sensitivity-weighted multicoil image reconstruction", Eq. (1),
  up to the unitary scale of the inverse transform (see :func:`eq1_factor`).
* :func:`E` is the forward model whose adjoint Eq. (1) is; :func:`A` is the
  composition E^H E (+ lambda I); :func:`cg` is conjugate gradients on it
  (CG-SENSE).  These follow the textbook definitions restated in the C file.
* :func:`rss` is the root-sum-of-squares reconstruction timed in the paper's
  Tables I and II (Section "Performance comparison with other frameworks").

Every function here is pinned by tests/test_oracle_*.py against brute
force, closed forms, invariants and library routines.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sense_oracle.c")
_LIB = os.path.join(_HERE, "libsense_oracle.so")

MAXITER, CONVERGED, EXACT, BREAKDOWN, NONFINITE = 0, 1, 2, 3, 4
STATUS_NAMES = {MAXITER: "maxiter", CONVERGED: "converged", EXACT: "exact",
                BREAKDOWN: "breakdown", NONFINITE: "nonfinite"}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp).  Always recompiles."""
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L = ctypes.c_long
        Ii = ctypes.c_int
        D = ctypes.c_double
        lib.or_fft1d.argtypes = [L, P, P, Ii]
        lib.or_dft1d_direct.argtypes = [L, P, P, Ii]
        lib.or_centred1d.argtypes = [L, P, P, Ii]
        lib.or_centred_nd.argtypes = [P, P, L, L, L, Ii]
        dims = [L, L, L, Ii, Ii, Ii]
        lib.or_E.argtypes = dims + [P, P, P, P]
        lib.or_EH.argtypes = dims + [P, P, P, P]
        lib.or_A.argtypes = dims + [P, P, P, D, P]
        lib.or_cg.argtypes = dims + [P, P, P, Ii, D, D, Ii, P, P, P, P]
        lib.or_rss.argtypes = [L, L, L, Ii, Ii, P, P]
        lib.or_set_threads.argtypes = [Ii]
        for f in ("or_set_threads", "or_fft1d", "or_dft1d_direct", "or_centred1d", "or_centred_nd",
                  "or_E", "or_EH", "or_A", "or_cg", "or_rss"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with code {rc}")


def fft1d(v, sign=-1):
    """Unnormalised DFT via the oracle's mixed-radix FFT (sign -1 forward)."""
    v = _c(v)
    out = np.empty_like(v)
    _check(_load().or_fft1d(v.size, _ptr(v), _ptr(out), sign), "fft1d")
    return out


def dft1d_direct(v, sign=-1):
    """Unnormalised DFT by the direct O(N^2) sum."""
    v = _c(v)
    out = np.empty_like(v)
    _check(_load().or_dft1d_direct(v.size, _ptr(v), _ptr(out), sign), "dft1d_direct")
    return out


def centred1d(v, direction=-1):
    """Centred unitary 1D transform: -1 = F_c, +1 = F_c^H."""
    v = _c(v)
    out = np.empty_like(v)
    _check(_load().or_centred1d(v.size, _ptr(v), _ptr(out), direction), "centred1d")
    return out


def centred_nd(img, direction=-1):
    """Centred unitary transform over all axes of a 1-3D image [Nz][Ny][Nx]."""
    img = _c(img)
    shape = img.shape
    nz, ny, nx = (1,) * (3 - img.ndim) + shape
    out = np.empty_like(img)
    _check(_load().or_centred_nd(_ptr(img), _ptr(out), nx, ny, nz, direction), "centred_nd")
    return out


def _geom(x_shape_tail, ndim):
    if ndim == 2:
        ny, nx = x_shape_tail[-2:]
        return nx, ny, 1
    nz, ny, nx = x_shape_tail[-3:]
    return nx, ny, nz


def _mask(mask, ny, nz):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.size != ny * nz:
        raise ValueError(f"mask has {m.size} entries, expected {ny * nz}")
    return m


def E(x, maps, mask, ndim=2):
    """Forward operator.  x: [B][(Nz)][Ny][Nx]; maps: [(B)][C][...]."""
    x = _c(x)
    nx, ny, nz = _geom(x.shape, ndim)
    nvox = nx * ny * nz
    batch = x.size // nvox
    maps = _c(maps)
    ncoils = maps.shape[-ndim - 1]
    shared = int(maps.size == ncoils * nvox)
    m = _mask(mask, ny, nz)
    y = np.empty((batch, ncoils) + x.shape[-ndim:], dtype=np.complex128)
    _check(_load().or_E(nx, ny, nz, ncoils, batch, shared, _ptr(x), _ptr(maps),
                        _ptr(m), _ptr(y)), "E")
    return y


def EH(y, maps, mask, ndim=2):
    """Adjoint operator.  y: [B][C][...]; returns [B][...]."""
    y = _c(y)
    nx, ny, nz = _geom(y.shape, ndim)
    nvox = nx * ny * nz
    ncoils = y.shape[-ndim - 1]
    batch = y.size // (nvox * ncoils)
    maps = _c(maps)
    shared = int(maps.size == ncoils * nvox)
    m = _mask(mask, ny, nz)
    x = np.empty((batch,) + y.shape[-ndim:], dtype=np.complex128)
    _check(_load().or_EH(nx, ny, nz, ncoils, batch, shared, _ptr(y), _ptr(maps),
                         _ptr(m), _ptr(x)), "EH")
    return x


def A(p, maps, mask, lam=0.0, ndim=2):
    """Normal operator E^H(E p) + lam p (composed)."""
    p = _c(p)
    nx, ny, nz = _geom(p.shape, ndim)
    nvox = nx * ny * nz
    batch = p.size // nvox
    maps = _c(maps)
    ncoils = maps.shape[-ndim - 1]
    shared = int(maps.size == ncoils * nvox)
    m = _mask(mask, ny, nz)
    q = np.empty((batch,) + p.shape[-ndim:], dtype=np.complex128)
    _check(_load().or_A(nx, ny, nz, ncoils, batch, shared, _ptr(p), _ptr(maps),
                        _ptr(m), float(lam), _ptr(q)), "A")
    return q


def cg(y, maps, mask, max_iter, tol=0.0, lam=0.0, ndim=2, vec32=False):
    """CG-SENSE.  Returns (x [B][...], iters [B], status [B], rho_hist [B][K+1]).

    vec32=True rounds every CG vector (b, q, x, r, p) to complex64 as it is
    produced, with the operator and the inner products in fp64: the error
    floor of complex64 storage alone."""
    y = _c(y)
    nx, ny, nz = _geom(y.shape, ndim)
    nvox = nx * ny * nz
    ncoils = y.shape[-ndim - 1]
    batch = y.size // (nvox * ncoils)
    maps = _c(maps)
    shared = int(maps.size == ncoils * nvox)
    m = _mask(mask, ny, nz)
    x = np.empty((batch,) + y.shape[-ndim:], dtype=np.complex128)
    iters = np.zeros(batch, dtype=np.int32)
    status = np.zeros(batch, dtype=np.int32)
    hist = np.zeros((batch, max_iter + 1), dtype=np.float64)
    _check(_load().or_cg(nx, ny, nz, ncoils, batch, shared, _ptr(y), _ptr(maps), _ptr(m),
                         int(max_iter), float(tol), float(lam), int(bool(vec32)), _ptr(x), _ptr(iters),
                         _ptr(status), _ptr(hist)), "cg")
    return x, iters, status, hist


def rss(y, ndim=2):
    """Root sum of squares of the coil images F_c^H y_c (no mask)."""
    y = _c(y)
    nx, ny, nz = _geom(y.shape, ndim)
    nvox = nx * ny * nz
    ncoils = y.shape[-ndim - 1]
    batch = y.size // (nvox * ncoils)
    out = np.empty((batch,) + y.shape[-ndim:], dtype=np.float64)
    _check(_load().or_rss(nx, ny, nz, ncoils, batch, _ptr(y), _ptr(out)), "rss")
    return out


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's parallel loops started from the calling
    thread (n <= 0 leaves it); returns the count in effect.  Timing only."""
    return int(_load().or_set_threads(int(n)))


def eq1_factor(nvox: int) -> float:
    """Eq. (1) with an unscaled inverse DFT of 1/N (numpy's ifft convention)
    equals nvox^(-1/2) times the unitary adjoint: M_eq1 = EH(y) / sqrt(nvox)."""
    return 1.0 / np.sqrt(nvox)
