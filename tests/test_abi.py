"""The C ABI without a GPU: the shared library loads, exports every function
declared in include/hntl.h, and rejects invalid arguments with the documented
status codes before touching the device."""
import ctypes as C
import re
from pathlib import Path

import pytest

from paper_2606_08813_amd import hntl

HEADER = Path(__file__).resolve().parents[1] / "include" / "hntl.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hntl_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "hntl_search" in names and "hntl_build" in names and len(names) >= 10
    L = hntl.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(hntl.EXPORTS), set(names) - set(hntl.EXPORTS)


def test_version_and_empty_error():
    assert "gfx950" in hntl.hntl_version()


def test_search_argument_validation_needs_no_device():
    L = hntl.lib()
    sp = hntl.hntl_search_params(0, 20, 10, 0, 0)
    assert L.hntl_search(None, None, 5, C.byref(sp), None, None, None) == hntl.HNTL_EINVAL
    assert "null" in hntl.hntl_last_error()


def test_create_argument_validation_needs_no_device():
    L = hntl.lib()
    out = C.c_void_p()
    nul = [None] * 7
    assert L.hntl_index_create(10, 4, 2, 2, *nul, 1, C.byref(out)) == hntl.HNTL_EINVAL
    dummy = C.c_void_p(1)
    args = [dummy] * 7
    assert L.hntl_index_create(10, 4, 11, 2, *args, 1, C.byref(out)) == hntl.HNTL_EINVAL   # G > N
    assert L.hntl_index_create(10, 4, 2, 5, *args, 1, C.byref(out)) == hntl.HNTL_EINVAL    # r > d
    assert L.hntl_index_create(100, 80, 2, 65, *args, 1, C.byref(out)) == hntl.HNTL_EUNSUPPORTED
    assert out.value is None


def test_build_argument_validation_needs_no_device():
    L = hntl.lib()
    out = C.c_void_p()
    p = hntl.hntl_build_params(0, 4, 0, 0, 0, 1, 0, None)
    assert L.hntl_build(C.c_void_p(1), 100, 8, C.byref(p), None, C.byref(out)) == hntl.HNTL_EINVAL   # G = 0
    p = hntl.hntl_build_params(4, 9, 0, 0, 0, 1, 0, None)
    assert L.hntl_build(C.c_void_p(1), 100, 8, C.byref(p), None, C.byref(out)) == hntl.HNTL_EINVAL   # r > d
    assert L.hntl_build(None, 100, 8, C.byref(p), None, C.byref(out)) == hntl.HNTL_EINVAL


def test_info_and_export_reject_null():
    L = hntl.lib()
    info = hntl.hntl_index_info()
    assert L.hntl_index_info_get(None, C.byref(info)) == hntl.HNTL_EINVAL
    assert L.hntl_index_export(None, *([None] * 7)) == hntl.HNTL_EINVAL
    L.hntl_index_free(None)


def test_append_save_load_argument_validation_needs_no_device(tmp_path):
    L = hntl.lib()
    out = C.c_void_p()
    p = hntl.hntl_append_params(0, 0, 0)
    assert L.hntl_index_append(None, None, 0, C.byref(p), None, C.byref(out)) == hntl.HNTL_EINVAL   # no base
    assert L.hntl_index_append(C.c_void_p(1), None, 0, C.byref(p), None, None) == hntl.HNTL_EINVAL  # no out
    assert L.hntl_index_save(None, str(tmp_path).encode()) == hntl.HNTL_EINVAL
    assert L.hntl_index_load(None, C.byref(out)) == hntl.HNTL_EINVAL
    # a directory without index files: an I/O error, found before any device call
    assert L.hntl_index_load(str(tmp_path / "none").encode(), C.byref(out)) == hntl.HNTL_EIO
    assert "meta.json" in hntl.hntl_last_error()
    (tmp_path / "meta.json").write_text('{"format": "something-else"}')
    assert L.hntl_index_load(str(tmp_path).encode(), C.byref(out)) == hntl.HNTL_EIO
    assert out.value is None
