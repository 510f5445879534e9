"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hologen.h declares, and rejects bad arguments with a
status code and a message before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2006_10509_amd import hologen as hg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hologen.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hg_plan_create", "hg_plan_destroy", "hg_workspace_bytes", "hg_propagate",
                     "hg_gs_iterate", "hg_ospr", "hg_error"):
        assert required in names
    assert set(names) == set(hg.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = hg.library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {hg.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", out), name


def create(**kw):
    d = dict(width=256, height=256, propagation=0, wavelength=0.0, pixel_pitch=0.0,
             distance=0.0, modulation=0, levels=0)
    d.update(kw)
    desc = hg.hg_plan_desc(**d)
    out = ctypes.c_void_p(12345)
    st = hg.library().hg_plan_create(ctypes.byref(desc), ctypes.byref(out))
    return st, out.value


@pytest.mark.parametrize("kw,status", [
    (dict(width=1), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(height=16384), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(width=1022), hg.HG_ERR_UNSUPPORTED_SIZE),          # factor 7 * 73
    (dict(width=4374), hg.HG_ERR_UNSUPPORTED_SIZE),          # 2 * 3^7: smooth, not compiled
    (dict(propagation=7), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(propagation=1, wavelength=532e-9, pixel_pitch=8e-6, distance=float("nan")), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(propagation=1, wavelength=-1.0, pixel_pitch=8e-6, distance=0.5), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(propagation=1, wavelength=532e-9, pixel_pitch=float("inf"), distance=0.5), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(modulation=0, levels=8), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(modulation=1, levels=1), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(modulation=1, levels=257), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(modulation=2, levels=4), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(modulation=9), hg.HG_ERR_INVALID_ARGUMENT),
    (dict(modulation=3, levels=4), hg.HG_ERR_INVALID_ARGUMENT),     # amplitude-only: continuous
])
def test_plan_create_rejects_bad_descriptors(kw, status):
    st, handle = create(**kw)
    assert st == status
    assert handle == 12345          # out untouched on failure
    msg = hg.hg_error(st)
    assert msg and ":" in msg        # detail attached for this thread's last status


def test_null_arguments_are_rejected_before_any_device_work():
    lib = hg.library()
    out = ctypes.c_void_p()
    assert lib.hg_plan_create(None, ctypes.byref(out)) == hg.HG_ERR_INVALID_ARGUMENT
    desc = hg.hg_plan_desc(256, 256, 0, 0, 0, 0, 0, 0)
    assert lib.hg_plan_create(ctypes.byref(desc), None) == hg.HG_ERR_INVALID_ARGUMENT
    assert lib.hg_propagate(None, 1, 1, 1, None, None) == hg.HG_ERR_INVALID_ARGUMENT
    assert lib.hg_gs_iterate(None, 1, None, 1, None, None, 3, 1, None) == hg.HG_ERR_INVALID_ARGUMENT
    assert lib.hg_ospr(None, 1, 1, 1, None, 1, None, 1, None) == hg.HG_ERR_INVALID_ARGUMENT
    assert lib.hg_gs_iterate_noalloc(None, 1, None, 1, None, None, 3, None) == hg.HG_ERR_INVALID_ARGUMENT
    assert lib.hg_workspace_bytes(None) == 0
    assert lib.hg_plan_destroy(None) == hg.HG_OK


def test_error_strings():
    for s, word in [(0, "success"), (1, "invalid"), (2, "unsupported"), (3, "memory"),
                    (4, "device"), (5, "internal"), (99, "unknown")]:
        assert word in hg.hg_error(s)


def test_supported_lengths():
    for n in (16, 256, 1024, 2048, 4096, 1080, 1920, 90, 120, 1280, 1536, 2160, 3840, 8192):
        assert hg.hg_length_supported(n)
    for n in (0, 1, 7, 1000, 8191, 16384):
        assert not hg.hg_length_supported(n)
