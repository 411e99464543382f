"""Host-side checks of the C ABI library (no GPU compute): it loads, exports
every entry point declared in include/mars.h, and rejects bad arguments."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mars.h")
LIB = os.path.join(ROOT, "paper_2410_20429_amd", "libmars.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mars_[a-z_0-9]+)\s*\(", txt)) - {"mars_alloc_fn", "mars_free_fn"})


@pytest.fixture(scope="module")
def libmars():
    if not os.path.exists(LIB):
        from paper_2410_20429_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for n in ["mars_create", "mars_scene_upload", "mars_render_iteration", "mars_update_counts",
              "mars_read_image", "mars_read_count_map"]:
        assert n in names


def test_library_exports_every_declared_symbol(libmars):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mars_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(libmars, n)


def test_null_arguments_rejected(libmars):
    libmars.mars_create.argtypes = [C.c_void_p, C.c_void_p]
    assert libmars.mars_create(None, None) == -1
    libmars.mars_render_iteration.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    assert libmars.mars_render_iteration(None, 0, None, None) == -1
    libmars.mars_destroy.argtypes = [C.c_void_p]
    assert libmars.mars_destroy(None) == -1
    libmars.mars_version.restype = C.c_char_p
    assert libmars.mars_version().startswith(b"mars")


def test_binding_names_match_header():
    from paper_2410_20429_amd import _capi
    for n in _declared():
        if n in ("mars_last_error", "mars_version", "mars_profile_kernel_name",
                 "mars_mlp_num_params"):
            continue
        assert n in _capi.SIGNATURES, n
        assert hasattr(_capi, n), n
