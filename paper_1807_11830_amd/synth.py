"""Seeded synthetic inputs for multicoil Cartesian MRI reconstruction.

The paper's case study reconstructs 2D cardiac cine data (16 frames of
160x160, 8 coils, fully sampled Cartesian k-space; Section "Case study: MRI
reconstruction", the cine workload paragraph after Tables I/II).  That data is
not available, so every workload here is built from seeded generators of the
same shape and structure:

* image: a sum of random ellipses (2D) or ellipsoids (3D) with intensities
  drawn from U[0.1, 1];
* coil sensitivities S_c: Gaussian bumps centred on evenly spaced points of
  the unit boundary circle, each with a linear phase, normalised pointwise so
  that sum_c |S_c|^2 = 1;
* sampling masks on the phase-encode axes (ky in 2D, (ky, kz) in 3D):
  regular R=2 with a fully sampled centre, or variable density with an exact
  line/point count;
* complex Gaussian noise with a stated per-component sigma.

This module only draws and shapes inputs.  It holds none of the
reconstruction arithmetic (no transforms, no operators), so both the CPU
oracle tests and the GPU path can consume it without sharing method code.
Every array is returned in numpy; complex images are complex128 (callers
cast to complex64 for the GPU).

Layouts (x = readout axis, fastest):
  image  [Nz][Ny][Nx]           (Nz omitted in 2D)
  maps   [C][Nz][Ny][Nx]
  mask2d [Ny] uint8, centred order (DC line at index Ny//2)
  mask3d [Nz][Ny] uint8, centred order (DC at (Nz//2, Ny//2))
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

SEED_PHANTOM = 11
SEED_MASK = 12
SEED_NOISE = 13
SEED_REQUESTS = 14


def _grid(n: int) -> np.ndarray:
    """Normalised coordinate (i - n/2) / (n/2) for i in [0, n)."""
    return (np.arange(n, dtype=np.float64) - n / 2.0) / (n / 2.0)


def phantom2d(n: int, n_ellipses: int = 10, seed: int = SEED_PHANTOM,
              ny: int | None = None) -> np.ndarray:
    """Sum of random ellipses on an ny x n grid, real valued, as complex128.

    Each ellipse draws, in order: centre (cx, cy) ~ U[-0.5, 0.5]^2, semi-axes
    a, b ~ U[0.1, 0.45], rotation ~ U[0, pi), intensity ~ U[0.1, 1].
    Overlapping ellipses add.
    """
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    u = _grid(n)[None, :]
    v = _grid(ny)[:, None]
    img = np.zeros((ny, n), dtype=np.float64)
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.5, 0.5, size=2)
        a, b = rng.uniform(0.1, 0.45, size=2)
        th = rng.uniform(0.0, np.pi)
        amp = rng.uniform(0.1, 1.0)
        du, dv = u - cx, v - cy
        xr = du * np.cos(th) + dv * np.sin(th)
        yr = -du * np.sin(th) + dv * np.cos(th)
        img += amp * (((xr / a) ** 2 + (yr / b) ** 2) <= 1.0)
    return img.astype(np.complex128)


def phantom3d(nx: int, ny: int, nz: int, n_ellipsoids: int = 10,
              seed: int = SEED_PHANTOM) -> np.ndarray:
    """Sum of random ellipsoids on an nz x ny x nx grid, as complex128.

    Each ellipsoid draws: centre ~ U[-0.5, 0.5]^3, semi-axes ~ U[0.1, 0.45]^3,
    rotation about z ~ U[0, pi), intensity ~ U[0.1, 1].
    """
    rng = np.random.default_rng(seed)
    u = _grid(nx)[None, None, :]
    v = _grid(ny)[None, :, None]
    w = _grid(nz)[:, None, None]
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    for _ in range(n_ellipsoids):
        cx, cy, cz = rng.uniform(-0.5, 0.5, size=3)
        a, b, c = rng.uniform(0.1, 0.45, size=3)
        th = rng.uniform(0.0, np.pi)
        amp = rng.uniform(0.1, 1.0)
        du, dv, dw = u - cx, v - cy, w - cz
        xr = du * np.cos(th) + dv * np.sin(th)
        yr = -du * np.sin(th) + dv * np.cos(th)
        vol += amp * (((xr / a) ** 2 + (yr / b) ** 2 + (dw / c) ** 2) <= 1.0)
    return vol.astype(np.complex128)


def _bump(u, v, w, centre, theta, width=0.6):
    d2 = (u - centre[0]) ** 2 + (v - centre[1]) ** 2 + (w - centre[2]) ** 2
    mag = np.exp(-d2 / (2.0 * width * width))
    phase = (np.pi / 2.0) * (u * np.cos(theta) + v * np.sin(theta)) + theta
    return mag * np.exp(1j * phase)


def coil_maps2d(n: int, ncoils: int, ny: int | None = None, rotation: float = 0.0) -> np.ndarray:
    """Gaussian-bump coil sensitivities [C][Ny][Nx] with sum_c |S_c|^2 = 1.

    Coil c sits at angle t = 2*pi*c/C + rotation on the unit circle;
    magnitude exp(-|r - r_c|^2 / (2 * 0.6^2)); phase (pi/2)(u cos t + v sin t) + t.
    A per-slice rotation gives every slice of a batch its own maps.
    """
    ny = n if ny is None else ny
    u = _grid(n)[None, :]
    v = _grid(ny)[:, None]
    maps = np.empty((ncoils, ny, n), dtype=np.complex128)
    for c in range(ncoils):
        t = 2.0 * np.pi * c / ncoils + rotation
        maps[c] = _bump(u, v, 0.0, (np.cos(t), np.sin(t), 0.0), t)
    maps /= np.sqrt(np.sum(np.abs(maps) ** 2, axis=0, keepdims=True))
    return maps


def coil_maps3d(nx: int, ny: int, nz: int, ncoils: int) -> np.ndarray:
    """3D coil sensitivities [C][Nz][Ny][Nx]: two rings of C/2 bumps at
    z = -0.5 and z = +0.5, the second ring rotated by pi/(C/2); normalised
    so that sum_c |S_c|^2 = 1 pointwise."""
    if ncoils % 2:
        raise ValueError("3D coil maps need an even coil count")
    half = ncoils // 2
    u = _grid(nx)[None, None, :]
    v = _grid(ny)[None, :, None]
    w = _grid(nz)[:, None, None]
    maps = np.empty((ncoils, nz, ny, nx), dtype=np.complex128)
    for ring, z in enumerate((-0.5, 0.5)):
        for j in range(half):
            t = 2.0 * np.pi * j / half + ring * np.pi / half
            maps[ring * half + j] = _bump(u, v, w, (np.cos(t), np.sin(t), z), t)
    maps /= np.sqrt(np.sum(np.abs(maps) ** 2, axis=0, keepdims=True))
    return maps


def mask_regular(n: int, step: int = 2, n_centre: int = 8) -> np.ndarray:
    """Lines k with k % step == 0 plus the n_centre lines around n/2."""
    m = np.zeros(n, dtype=np.uint8)
    m[::step] = 1
    m[n // 2 - n_centre // 2: n // 2 + n_centre // 2] = 1
    return m


def _weighted_topk(keys_u: np.ndarray, weights: np.ndarray, k: int,
                   excluded: np.ndarray) -> np.ndarray:
    """Efraimidis-Spirakis weighted sampling without replacement: key
    u^(1/w), keep the k largest; ties go to the lower flat index."""
    with np.errstate(divide="ignore"):
        expo = np.where(weights > 0, 1.0 / np.where(weights > 0, weights, 1.0), np.inf)
        keys = np.where(weights > 0, keys_u ** expo, 0.0)
    keys = np.where(excluded, -1.0, keys)
    order = np.lexsort((np.arange(keys.size), -keys))
    return order[:k]


def mask_variable_density(n: int, accel: float, n_centre: int = 24,
                          seed: int = SEED_MASK) -> np.ndarray:
    """Phase-encode mask with exactly round(n / accel) lines: n_centre fully
    sampled centre lines (clipped to the line budget) plus weighted sampling
    without replacement of the rest, weight (1 - |k - n/2| / (n/2))^2."""
    n_lines = int(round(n / accel))
    n_centre = min(n_centre, n_lines)
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    k = np.arange(n, dtype=np.float64)
    w = np.clip(1.0 - np.abs(k - n / 2.0) / (n / 2.0), 0.0, None) ** 2
    m = np.zeros(n, dtype=np.uint8)
    lo = n // 2 - n_centre // 2
    m[lo: lo + n_centre] = 1
    rest = n_lines - n_centre
    if rest > 0:
        pick = _weighted_topk(u, w, rest, m.astype(bool))
        m[pick] = 1
    assert int(m.sum()) == n_lines
    return m


def mask_variable_density_2d(ny: int, nz: int, accel: float, centre=(32, 32),
                             seed: int = SEED_MASK) -> np.ndarray:
    """(kz, ky) point mask [Nz][Ny] with exactly round(ny*nz/accel) points,
    a fully sampled centre block of centre[0] (ky) x centre[1] (kz) points,
    and radial weight (1 - r)^2, r = normalised distance from the centre."""
    n_pts = int(round(ny * nz / accel))
    rng = np.random.default_rng(seed)
    u = rng.random(ny * nz)
    kz = (np.arange(nz, dtype=np.float64) - nz / 2.0) / (nz / 2.0)
    ky = (np.arange(ny, dtype=np.float64) - ny / 2.0) / (ny / 2.0)
    r = np.sqrt(kz[:, None] ** 2 + ky[None, :] ** 2)
    w = (np.clip(1.0 - r, 0.0, None) ** 2).ravel()
    m = np.zeros((nz, ny), dtype=np.uint8)
    cy, cz = min(centre[0], ny), min(centre[1], nz)
    m[nz // 2 - cz // 2: nz // 2 - cz // 2 + cz, ny // 2 - cy // 2: ny // 2 - cy // 2 + cy] = 1
    rest = n_pts - int(m.sum())
    if rest > 0:
        pick = _weighted_topk(u, w, rest, m.ravel().astype(bool))
        m.ravel()[pick] = 1
    assert int(m.sum()) == n_pts
    return m


def complex_noise(shape, sigma: float = 1e-3, seed: int = SEED_NOISE) -> np.ndarray:
    """Complex Gaussian noise, sigma per real component."""
    rng = np.random.default_rng(seed)
    return sigma * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def complex_normal(shape, seed: int) -> np.ndarray:
    """Complex standard normal (unit variance per real component)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# Workload descriptions (sizes only; no arithmetic of the method)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload2D:
    name: str
    n: int           # Nx = Ny
    ncoils: int
    batch: int
    iters: int
    mask: str        # "regular" or "vd"
    accel: float
    n_centre: int

    def mask_array(self, seed: int = SEED_MASK) -> np.ndarray:
        if self.mask == "regular":
            return mask_regular(self.n, 2, self.n_centre)
        return mask_variable_density(self.n, self.accel, self.n_centre, seed)


# Plain CG-SENSE, single 64x64 slice, 4 coils, R=2 regular + 8 centre lines, 20 iterations.
SMALL_64 = Workload2D("cgsense_64x64_c4_r2_k20", 64, 4, 1, 20, "regular", 2.0, 8)
# Plain CG-SENSE, 256x256 slice, 12 coils, VD R=4 with 24 centre lines, 30 iterations.
SLICE_256 = Workload2D("cgsense_256x256_c12_vdr4_k30", 256, 12, 1, 30, "vd", 4.0, 24)
# Precision workload: 384x384, 32 coils, batch 8, VD R=4, 40 iterations.
PREC_384 = Workload2D("cgsense_384x384_c32_b8_vdr4_k40", 384, 32, 8, 40, "vd", 4.0, 24)


def slice_inputs(w: Workload2D, batch: int | None = None, seed: int = SEED_PHANTOM,
                 per_slice_maps: bool = False):
    """Image batch [B][N][N], maps and mask [N] for a 2D workload.

    Batch element b uses phantom seed `seed + b`, so slices differ.  Maps are
    [C][N][N] (shared), or [B][C][N][N] with per_slice_maps, slice b rotated
    by 2*pi*b / (B*C).
    """
    b = w.batch if batch is None else batch
    imgs = np.stack([phantom2d(w.n, seed=seed + i) for i in range(b)])
    if per_slice_maps:
        maps = np.stack([coil_maps2d(w.n, w.ncoils, rotation=2.0 * np.pi * i / (b * w.ncoils))
                         for i in range(b)])
    else:
        maps = coil_maps2d(w.n, w.ncoils)
    return imgs, maps, w.mask_array()


def request_stream(n_requests: int = 512, rate: float = 1.0,
                   seed: int = SEED_REQUESTS,
                   sizes=(128, 192, 256, 320), coils=(8, 16, 32),
                   accels=(2, 3, 4)):
    """Serving workload: Poisson arrivals (exponential gaps of mean 1/rate)
    with size, coil count and acceleration drawn uniformly per request.
    Returns a list of dicts with per-request sub-seeds from SeedSequence."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    children = ss.spawn(n_requests)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        out.append(dict(id=i, arrival=t,
                        n=int(rng.choice(sizes)), ncoils=int(rng.choice(coils)),
                        accel=int(rng.choice(accels)),
                        seed=int(children[i].generate_state(1)[0])))
    return out
