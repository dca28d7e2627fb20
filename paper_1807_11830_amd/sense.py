"""ctypes binding of the gfx950 CG-SENSE library (include/sense.h).

Argument marshalling only: torch supplies device memory and the current
stream, every operator step runs in the HIP kernels of libsense_gfx950.so.
There is no fallback: if the library is missing or a call fails, a
:class:`SenseError` is raised.

Names follow the operator notation of the paper (arXiv 1807.11830, Eq. (1)
and the multicoil model around it): sensitivity maps S, k-space y, image x,
sampling mask M, and the operators E, E^H (``EH``) and E^H E (``EHE``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsense_gfx950.so")

C64, BF16X2, FP16X2 = 0, 1, 2
STORAGE = {"c64": C64, "bf16": BF16X2, "fp16": FP16X2}
MAXITER, CONVERGED, EXACT, BREAKDOWN, NONFINITE = 0, 1, 2, 3, 4
STATUS_NAMES = {MAXITER: "maxiter", CONVERGED: "converged", EXACT: "exact",
                BREAKDOWN: "breakdown", NONFINITE: "nonfinite"}
ERRORS = {1: "invalid argument", 2: "unsupported", 3: "out of memory", 4: "device error",
          5: "bad state"}

# Lengths with compiled transforms (Ny always; Nx for E, E^H and CG).
SUPPORTED_LENGTHS = (8, 16, 32, 48, 64, 80, 96, 128, 160, 192, 256, 320, 384)


class SenseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sense error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("ncoils", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("maps_storage", ctypes.c_int32), ("kspace_storage", ctypes.c_int32),
                ("maps_shared", ctypes.c_int32), ("kspace_compact", ctypes.c_int32)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iters_run", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rho0", ctypes.c_double), ("rho_final", ctypes.c_double)]


ABI_FUNCTIONS = ("sense_plan_device_bytes", "sense_plan_create", "sense_plan_destroy",
                 "sense_apply_E", "sense_apply_EH", "sense_apply_EHE", "sense_apply_rss", "sense_cg_solve",
                 "sense_plan_cg_info", "sense_plan_set_profiling", "sense_plan_profile",
                 "sense_plan_set_graphs", "sense_plan_set_maps", "sense_plan_set_coil_groups",
                 "sense_plan_coil_groups", "sense_engine_create", "sense_engine_destroy",
                 "sense_engine_admit", "sense_engine_step", "sense_engine_poll", "sense_engine_stats",
                 "sense_engine_sync", "sense_last_error", "sense_version", "sense_cg_solve_static")

_lib = None


def lib():
    """Load the HIP library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SenseError(4, f"{LIB_PATH} is missing: build it with "
                            "`python -m paper_1807_11830_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.sense_plan_device_bytes.argtypes = [ctypes.POINTER(Desc)]
    L.sense_plan_device_bytes.restype = ctypes.c_size_t
    L.sense_plan_create.argtypes = [ctypes.POINTER(Desc), P, P, P, ctypes.POINTER(P)]
    L.sense_plan_destroy.argtypes = [P]
    L.sense_apply_E.argtypes = [P, P, P, P]
    L.sense_apply_EH.argtypes = [P, P, P, P]
    L.sense_apply_EHE.argtypes = [P, P, P, D, P]
    L.sense_apply_rss.argtypes = [P, P, P, P]
    L.sense_cg_solve.argtypes = [P, P, P, I32, D, D, P, P, P]
    L.sense_cg_solve_static.argtypes = [ctypes.POINTER(Desc), P, P, P, P, I32, D, D, P, P, P]
    L.sense_plan_cg_info.argtypes = [P, P, P]
    L.sense_plan_set_profiling.argtypes = [P, I32]
    L.sense_plan_set_graphs.argtypes = [P, I32]
    L.sense_plan_set_maps.argtypes = [P, P]
    L.sense_plan_set_coil_groups.argtypes = [P, I32]
    L.sense_plan_coil_groups.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.sense_plan_profile.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(D)]
    L.sense_engine_create.argtypes = [ctypes.c_size_t, I32, ctypes.POINTER(P)]
    L.sense_engine_destroy.argtypes = [P]
    L.sense_engine_admit.argtypes = [P, P, P, P, I32, D, D, ctypes.c_size_t, P, ctypes.POINTER(I32)]
    L.sense_engine_step.argtypes = [P, ctypes.POINTER(I32)]
    L.sense_engine_poll.argtypes = [P, ctypes.POINTER(I32), I32, ctypes.POINTER(I32)]
    L.sense_engine_stats.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(I32), ctypes.POINTER(I64)]
    L.sense_engine_sync.argtypes = [P]
    L.sense_last_error.argtypes = []
    L.sense_last_error.restype = ctypes.c_char_p
    L.sense_version.argtypes = []
    L.sense_version.restype = ctypes.c_char_p
    for f in ABI_FUNCTIONS:
        if f not in ("sense_plan_device_bytes", "sense_last_error", "sense_version"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise SenseError(rc, lib().sense_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def to_storage(a: torch.Tensor, storage: str) -> torch.Tensor:
    """Complex tensor -> the library's interleaved storage (input marshalling).

    c64 returns a contiguous complex64 tensor; bf16/fp16 return the
    interleaved (re, im) 16-bit pairs with round-to-nearest-even."""
    a = a.to(torch.complex64).contiguous()
    if storage == "c64":
        return a
    dt = torch.bfloat16 if storage == "bf16" else torch.float16
    return torch.view_as_real(a).to(dt).contiguous()


def from_storage(a: torch.Tensor, storage: str) -> torch.Tensor:
    if storage == "c64":
        return a
    return torch.view_as_complex(a.to(torch.float32).contiguous())


def device_bytes(nx, ny, ncoils, batch, nz=1, ndim=None, maps_storage="c64", kspace_storage="c64",
                 maps_shared=True) -> int:
    """Device bytes of a plan (sense_plan_device_bytes); 0 if unsupported."""
    ndim = (3 if nz > 1 else 2) if ndim is None else ndim
    d = Desc(ndim, nx, ny, nz, ncoils, batch, STORAGE[maps_storage], STORAGE[kspace_storage],
             int(maps_shared))
    return int(lib().sense_plan_device_bytes(ctypes.byref(d)))


@dataclass
class CgResult:
    x: torch.Tensor
    iters: np.ndarray
    status: np.ndarray
    rho0: np.ndarray
    rho_final: np.ndarray
    rho_hist: torch.Tensor | None


class Plan:
    """A SENSE operator instance: maps, mask and sizes fixed at creation.

    maps: complex tensor on the GPU, [C][Ny][Nx] (shared by every batch
          element) or [B][C][Ny][Nx]; converted to ``maps_storage`` once.
    mask: uint8 array of Ny entries in centred order (DC at Ny // 2).
    kspace_compact: k-space holds only the sampled lines, [B][C][L][Nx].
    """

    def __init__(self, maps: torch.Tensor, mask, batch: int = 1, maps_storage: str = "c64",
                 kspace_storage: str = "c64", ndim: int | None = None, stream=None,
                 kspace_compact: bool = False):
        if not maps.is_cuda:
            raise SenseError(1, "maps must be a GPU tensor")
        m = np.asarray(mask if not torch.is_tensor(mask) else mask.cpu().numpy())
        if ndim is None:
            ndim = 3 if m.ndim == 2 else 2
        if ndim not in (2, 3):
            raise SenseError(1, "ndim must be 2 or 3")
        packed = maps.dtype in (torch.bfloat16, torch.float16)
        mdim = maps.dim() - (1 if packed else 0)  # 16-bit pairs carry a trailing 2
        if mdim == ndim + 1:
            shared = True
            dims = tuple(maps.shape[:mdim])
        elif mdim == ndim + 2:
            shared = False
            if maps.shape[0] != batch:
                raise SenseError(1, "maps batch dimension must equal batch")
            dims = tuple(maps.shape[1:mdim])
        else:
            raise SenseError(1, f"maps must be [C]{'[Nz]' if ndim == 3 else ''}[Ny][Nx] or [B][C]...")
        ncoils = dims[0]
        nz, ny, nx = (1,) + dims[1:] if ndim == 2 else dims[1:]
        self.ndim = ndim
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.ncoils, self.batch = int(ncoils), int(batch)
        self.maps_storage, self.kspace_storage = maps_storage, kspace_storage
        self.maps_shared = shared
        self.device = maps.device
        self._maps = maps.contiguous() if packed else to_storage(maps, maps_storage)
        m = np.ascontiguousarray(m, dtype=np.uint8)
        if m.size != self.ny * self.nz:
            raise SenseError(1, f"mask needs {self.ny * self.nz} entries")
        self.mask = m
        self.kspace_compact = bool(kspace_compact)
        self.nlines = int(np.count_nonzero(m))
        self.desc = Desc(ndim, self.nx, self.ny, self.nz, self.ncoils, self.batch, STORAGE[maps_storage],
                         STORAGE[kspace_storage], int(shared), int(self.kspace_compact))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().sense_plan_create(ctypes.byref(self.desc), _ptr(self._maps),
                                           m.ctypes.data_as(ctypes.c_void_p), _stream(stream),
                                           ctypes.byref(h)))
        self._h = h

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            with torch.cuda.device(self.device):
                _check(lib().sense_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- shapes ------------------------------------------------------------
    @property
    def grid(self):
        return (self.ny, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def image_shape(self):
        return (self.batch,) + self.grid

    @property
    def kspace_shape(self):
        if self.kspace_compact:
            return (self.batch, self.ncoils, self.nlines, self.nx)
        return (self.batch, self.ncoils) + self.grid

    @property
    def kspace_numel(self):
        n = 1
        for d in self.kspace_shape:
            n *= d
        return n

    @property
    def nvox(self):
        return self.nx * self.ny * self.nz

    def _img(self, t: torch.Tensor, name: str):
        if t.dtype != torch.complex64 or not t.is_contiguous() or t.device != self.device:
            raise SenseError(1, f"{name} must be a contiguous complex64 tensor on {self.device}")
        if t.numel() != self.batch * self.nvox:
            raise SenseError(1, f"{name} must have {self.image_shape} elements")
        return t

    def _ksp(self, t: torch.Tensor, name: str):
        if self.kspace_storage == "c64":
            ok = t.dtype == torch.complex64 and t.numel() == self.kspace_numel
        else:
            dt = torch.bfloat16 if self.kspace_storage == "bf16" else torch.float16
            ok = t.dtype == dt and t.numel() == 2 * self.kspace_numel
        if not ok or not t.is_contiguous() or t.device != self.device:
            raise SenseError(1, f"{name} must be contiguous k-space in {self.kspace_storage} storage")
        return t

    def new_kspace(self):
        if self.kspace_storage == "c64":
            return torch.empty(self.kspace_shape, dtype=torch.complex64, device=self.device)
        dt = torch.bfloat16 if self.kspace_storage == "bf16" else torch.float16
        return torch.empty(self.kspace_shape + (2,), dtype=dt, device=self.device)

    # -- operators -----------------------------------------------------------
    def E(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        x = self._img(x, "x")
        y = self.new_kspace() if out is None else self._ksp(out, "out")
        with torch.cuda.device(self.device):
            _check(lib().sense_apply_E(self._h, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def EH(self, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        y = self._ksp(y, "y")
        x = torch.empty(self.image_shape, dtype=torch.complex64, device=self.device) if out is None \
            else self._img(out, "out")
        with torch.cuda.device(self.device):
            _check(lib().sense_apply_EH(self._h, _ptr(y), _ptr(x), _stream(stream)))
        return x

    def rss(self, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Root-sum-of-squares image (float32 [B][...]) of the masked k-space."""
        y = self._ksp(y, "y")
        if out is None:
            img = torch.empty(self.image_shape, dtype=torch.float32, device=self.device)
        else:
            if out.dtype != torch.float32 or tuple(out.shape) != tuple(self.image_shape) or not out.is_contiguous():
                raise SenseError(1, f"out must be a contiguous float32 tensor of shape {tuple(self.image_shape)}")
            img = out
        with torch.cuda.device(self.device):
            _check(lib().sense_apply_rss(self._h, _ptr(y), _ptr(img), _stream(stream)))
        return img

    def EHE(self, p: torch.Tensor, lam: float = 0.0, out: torch.Tensor | None = None,
            stream=None) -> torch.Tensor:
        p = self._img(p, "p")
        q = torch.empty_like(p) if out is None else self._img(out, "out")
        with torch.cuda.device(self.device):
            _check(lib().sense_apply_EHE(self._h, _ptr(p), _ptr(q), float(lam), _stream(stream)))
        return q

    def cg(self, y: torch.Tensor, max_iter: int, tol: float = 0.0, lam: float = 0.0,
           out: torch.Tensor | None = None, history: bool = False, stream=None,
           sync: bool = True) -> CgResult:
        """CG-SENSE.  With sync=False the info arrays are left unread (None)."""
        y = self._ksp(y, "y")
        x = torch.empty(self.image_shape, dtype=torch.complex64, device=self.device) if out is None \
            else self._img(out, "out")
        hist = torch.zeros((self.batch, max_iter + 1), dtype=torch.float64, device=self.device) \
            if history else None
        with torch.cuda.device(self.device):
            _check(lib().sense_cg_solve(self._h, _ptr(y), _ptr(x), int(max_iter), float(tol),
                                        float(lam), None,
                                        _ptr(hist) if hist is not None else None, _stream(stream)))
            if not sync:
                return CgResult(x, None, None, None, None, hist)
            info = (CgInfo * self.batch)()
            _check(lib().sense_plan_cg_info(self._h, ctypes.cast(info, ctypes.c_void_p),
                                            _stream(stream)))
        return CgResult(x, np.array([i.iters_run for i in info]), np.array([i.status for i in info]),
                        np.array([i.rho0 for i in info]), np.array([i.rho_final for i in info]), hist)

    def set_maps(self, maps: torch.Tensor):
        """Rebind to another map buffer of the same shape and storage."""
        m = maps.contiguous() if maps.dtype in (torch.bfloat16, torch.float16) \
            else to_storage(maps, self.maps_storage)
        if m.numel() != self._maps.numel() or m.dtype != self._maps.dtype:
            raise SenseError(1, "maps must keep the plan's shape and storage")
        with torch.cuda.device(self.device):
            _check(lib().sense_plan_set_maps(self._h, _ptr(m)))
        self._maps = m

    def set_coil_groups(self, groups: int):
        """Force G coil groups (1 = no split; 0 = the plan's automatic choice)."""
        _check(lib().sense_plan_set_coil_groups(self._h, int(groups)))

    def coil_groups(self):
        """(current G, largest G the plan's workspace holds)."""
        g, gm = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sense_plan_coil_groups(self._h, ctypes.byref(g), ctypes.byref(gm)))
        return g.value, gm.value

    def set_graphs(self, on: bool):
        """Replay whole solves from a captured HIP graph (default on)."""
        _check(lib().sense_plan_set_graphs(self._h, int(bool(on))))

    # -- profiling -------------------------------------------------------------
    def set_profiling(self, on: bool):
        _check(lib().sense_plan_set_profiling(self._h, int(bool(on))))

    def profile(self):
        """(number of timed E^H E launches, total ms); clears the record."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        with torch.cuda.device(self.device):
            _check(lib().sense_plan_profile(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)


def cg_solve_static(maps: torch.Tensor, mask, y: torch.Tensor, x: torch.Tensor, max_iter: int,
                    tol: float = 0.0, lam: float = 0.0, batch: int = 1, maps_storage: str = "c64",
                    kspace_storage: str = "c64", info: torch.Tensor | None = None,
                    rho_hist: torch.Tensor | None = None, stream=None, kspace_compact: bool = False) -> None:
    """CG-SENSE of a 2D problem without a plan (sense_cg_solve_static).

    The library allocates nothing: its tables and work vectors live in a
    static device array (64 MiB per GPU).  maps [C][Ny][Nx] or
    [B][C][Ny][Nx] already in ``maps_storage`` (complex64, or interleaved
    16-bit pairs with a trailing 2), mask uint8 [Ny] centred, y k-space in
    ``kspace_storage``, x the complex64 [B][Ny][Nx] output; info (optional)
    a device uint8 tensor of 24 * B bytes receiving sense_cg_info per
    problem, rho_hist (optional) float64 [B][max_iter + 1].  With
    kspace_compact, y holds the sampled lines only ([B][C][L][Nx]).  Calls
    on one GPU must not overlap."""
    packed = maps.dtype in (torch.bfloat16, torch.float16)
    mdim = maps.dim() - (1 if packed else 0)
    if mdim == 3:
        shared, (ncoils, ny, nx) = 1, tuple(maps.shape[:3])
    elif mdim == 4:
        shared, (ncoils, ny, nx) = 0, tuple(maps.shape[1:4])
    else:
        raise SenseError(1, "maps must be [C][Ny][Nx] or [B][C][Ny][Nx]")
    m = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
    if m.size != ny:
        raise SenseError(1, f"mask needs {ny} entries")
    for t, name in ((maps, "maps"), (y, "y"), (x, "x")):
        if not t.is_cuda or not t.is_contiguous():
            raise SenseError(1, f"{name} must be a contiguous GPU tensor")
    if x.dtype != torch.complex64 or x.numel() != batch * ny * nx:
        raise SenseError(1, "x must be complex64 [B][Ny][Nx]")
    if info is not None and (info.dtype != torch.uint8 or info.numel() != 24 * batch or not info.is_cuda):
        raise SenseError(1, "info must be a device uint8 tensor of 24 * batch bytes")
    if rho_hist is not None and (rho_hist.dtype != torch.float64 or rho_hist.numel() != batch * (max_iter + 1)):
        raise SenseError(1, "rho_hist must be float64 [B][max_iter + 1]")
    d = Desc(2, int(nx), int(ny), 1, int(ncoils), int(batch), STORAGE[maps_storage], STORAGE[kspace_storage],
             shared, int(bool(kspace_compact)))
    with torch.cuda.device(x.device):
        _check(lib().sense_cg_solve_static(ctypes.byref(d), _ptr(maps), m.ctypes.data_as(ctypes.c_void_p),
                                           _ptr(y), _ptr(x), int(max_iter), float(tol), float(lam),
                                           _ptr(info) if info is not None else None,
                                           _ptr(rho_hist) if rho_hist is not None else None, _stream(stream)))


class Engine:
    """Continuous-batching CG engine (sense_engine_*): a slot table of
    single-slice solves advanced together, one CG iteration per step."""

    def __init__(self, budget_bytes: int, max_slots: int, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.max_slots = int(max_slots)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().sense_engine_create(int(budget_bytes), self.max_slots, ctypes.byref(h)))
        self._h = h
        self._done = (ctypes.c_int32 * self.max_slots)()
        # plan, y and x of every admitted slot, held until poll reports it:
        # the engine's streams read and write them, and torch's allocator
        # must not hand their memory to another tensor before then
        self._held = {}

    def admit(self, plan: Plan, y: torch.Tensor, x: torch.Tensor, max_iter: int, tol: float = 0.0,
              lam: float = 0.0, footprint: int = 0, stream=None):
        """Slot index, or None when no slot or budget is free right now.

        The engine orders the solve after the work already enqueued on
        ``stream`` (default: torch's current stream), where y was produced."""
        plan._ksp(y, "y")
        plan._img(x, "x")
        slot = ctypes.c_int32(-1)
        with torch.cuda.device(self.device):
            rc = lib().sense_engine_admit(self._h, plan._h, _ptr(y), _ptr(x), int(max_iter), float(tol),
                                          float(lam), int(footprint), _stream(stream), ctypes.byref(slot))
        if rc == 5:  # SENSE_ERR_STATE: full or over budget -> try again later
            msg = lib().sense_last_error().decode()
            if "no free slot" in msg or "budget" in msg:
                return None
        _check(rc)
        self._held[int(slot.value)] = (plan, y, x)
        return int(slot.value)

    def step(self) -> int:
        n = ctypes.c_int32(0)
        with torch.cuda.device(self.device):
            _check(lib().sense_engine_step(self._h, ctypes.byref(n)))
        return int(n.value)

    def poll(self):
        n = ctypes.c_int32(0)
        with torch.cuda.device(self.device):
            _check(lib().sense_engine_poll(self._h, self._done, self.max_slots, ctypes.byref(n)))
        done = [int(self._done[i]) for i in range(n.value)]
        for slot in done:
            self._held.pop(slot, None)
        return done

    def stats(self):
        used, budget = ctypes.c_size_t(0), ctypes.c_size_t(0)
        active, steps = ctypes.c_int32(0), ctypes.c_int64(0)
        _check(lib().sense_engine_stats(self._h, ctypes.byref(used), ctypes.byref(budget),
                                        ctypes.byref(active), ctypes.byref(steps)))
        return dict(used=used.value, budget=budget.value, active=active.value, steps=steps.value)

    def sync(self):
        with torch.cuda.device(self.device):
            _check(lib().sense_engine_sync(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            with torch.cuda.device(self.device):
                _check(lib().sense_engine_destroy(self._h))  # waits for the engine's streams
            self._h = ctypes.c_void_p()
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
