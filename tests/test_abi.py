"""C ABI of the HIP library, checked on the CPU (no GPU calls).

The library must load, export every function include/sense.h declares, and
reject invalid descriptors with the right status and a message before any
device work.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1807_11830_amd import sense

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sense.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SENSE_API\s+[\w\s\*]+?\b(sense_\w+)\s*\(", text)))


def test_header_declares_the_abi():
    names = _declared()
    assert set(names) == set(sense.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", sense.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for name in _declared():
        assert name in exported, name
        assert hasattr(sense.lib(), name)
    # nothing but the C ABI is exported from the library's own code
    assert {n for n in exported if n.startswith("sense")} == set(_declared())


def test_version():
    assert sense.lib().sense_version().decode().startswith("sense-gfx950")


def _desc(**kw):
    d = dict(ndim=2, nx=64, ny=64, nz=1, ncoils=4, batch=1, maps_storage=0, kspace_storage=0,
             maps_shared=1, kspace_compact=0)
    d.update(kw)
    return sense.Desc(**d)


def test_device_bytes():
    L = sense.lib()
    d = _desc(nx=256, ny=256, ncoils=12, batch=3)
    nb = L.sense_plan_device_bytes(ctypes.byref(d))
    nvox = 256 * 256
    # 16 column tiles x 3 slices = 48 blocks < 512: the plan splits the 12
    # coils into min(ceil(512 / 48), 12 / 2, 16) = 6 groups
    G = 6
    # workspace + r, p, q and the second r, p + the group partials
    vecs = 8 * nvox * 3 * (12 + 5 + G)
    assert vecs <= nb < vecs + (1 << 20)
    d = _desc(nx=256, ny=256, ncoils=12, batch=32)  # 512 blocks: no split
    nb = L.sense_plan_device_bytes(ctypes.byref(d))
    vecs = 8 * nvox * 32 * (12 + 3)
    assert vecs <= nb < vecs + (1 << 20)
    for bad in (dict(ndim=4), dict(nx=0), dict(ny=100), dict(nz=2), dict(ncoils=0),
                dict(maps_storage=7), dict(ndim=3, nz=7)):
        assert L.sense_plan_device_bytes(ctypes.byref(_desc(**bad))) == 0, bad


@pytest.mark.parametrize("kw,code,word", [
    (dict(ndim=1), 1, "ndim"),
    (dict(nx=0), 1, "sizes"),
    (dict(ny=100), 2, "ny=100"),
    (dict(ndim=3, nz=12), 2, "nz=12"),
    (dict(nz=2), 1, "nz"),
    (dict(kspace_storage=5), 1, "storage"),
    (dict(maps_shared=2), 1, "maps_shared"),
    (dict(kspace_compact=3), 1, "kspace_compact"),
])
def test_plan_create_rejects(kw, code, word):
    L = sense.lib()
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(1)
    mask = (ctypes.c_uint8 * 64)()
    rc = L.sense_plan_create(ctypes.byref(_desc(**kw)), dummy, ctypes.cast(mask, ctypes.c_void_p),
                             None, ctypes.byref(h))
    assert rc == code
    assert word in L.sense_last_error().decode()
    assert h.value is None


def test_null_arguments():
    L = sense.lib()
    h = ctypes.c_void_p()
    mask = (ctypes.c_uint8 * 64)()
    assert L.sense_plan_create(None, ctypes.c_void_p(256), ctypes.cast(mask, ctypes.c_void_p), None,
                               ctypes.byref(h)) == 1
    assert L.sense_plan_create(ctypes.byref(_desc()), None, ctypes.cast(mask, ctypes.c_void_p), None,
                               ctypes.byref(h)) == 1
    assert "d_maps" in L.sense_last_error().decode()
    assert L.sense_plan_create(ctypes.byref(_desc()), ctypes.c_void_p(256), None, None,
                               ctypes.byref(h)) == 1
    assert "h_mask" in L.sense_last_error().decode()
    assert L.sense_plan_create(ctypes.byref(_desc()), ctypes.c_void_p(256),
                               ctypes.cast(mask, ctypes.c_void_p), None, None) == 1
    for f, args in (("sense_apply_E", (None, None, None, None)),
                    ("sense_apply_EH", (None, None, None, None)),
                    ("sense_apply_EHE", (None, None, None, 0.0, None)),
                    ("sense_apply_rss", (None, None, None, None)),
                    ("sense_cg_solve", (None, None, None, 1, 0.0, 0.0, None, None, None)),
                    ("sense_plan_destroy", (None,)),
                    ("sense_plan_set_profiling", (None, 1)),
                    ("sense_plan_set_coil_groups", (None, 1)),
                    ("sense_plan_coil_groups", (None, None, None))):
        assert getattr(L, f)(*args) == 1, f
        assert "plan is NULL" in L.sense_last_error().decode()


def test_misaligned_maps_rejected():
    """Device buffers must be 16-byte aligned; the maps pointer is checked
    before any device call, so this runs without a GPU."""
    L = sense.lib()
    h = ctypes.c_void_p()
    mask = (ctypes.c_uint8 * 64)(*([1] * 64))
    assert L.sense_plan_create(ctypes.byref(_desc()), ctypes.c_void_p(256 + 8),
                               ctypes.cast(mask, ctypes.c_void_p), None, ctypes.byref(h)) == 1
    assert "d_maps must be 16-byte aligned" in L.sense_last_error().decode()
    assert not h.value
    assert L.sense_cg_solve_static(ctypes.byref(_desc()), ctypes.c_void_p(256 + 4),
                                   ctypes.cast(mask, ctypes.c_void_p), ctypes.c_void_p(512),
                                   ctypes.c_void_p(1024), 5, 0.0, 0.0, None, None, None) == 1
    assert "d_maps must be 16-byte aligned" in L.sense_last_error().decode()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sense, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sense, "_lib", None)
    with pytest.raises(sense.SenseError, match="no CPU fallback"):
        sense.lib()
