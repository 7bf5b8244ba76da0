"""CPU checks of the boundary: the C-ABI library loads and exports every symbol the header
declares, and the Python binding marshals the same names.  No compute call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nrrs.h")).read()
    decl = r"^(?:int32_t|void|const char\*)\s+(nrrs_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2510_07868_amd import nrrs
    if not os.path.exists(nrrs.LIB_PATH):
        from paper_2510_07868_amd import build
        build.build()
    return nrrs.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("nrrs_create", "nrrs_upload_scene", "nrrs_render", "nrrs_train_step", "nrrs_read_image",
                 "nrrs_debug_rrs_expand", "nrrs_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_binding_covers_the_exports(lib):
    from paper_2510_07868_amd import nrrs
    assert sorted(nrrs.EXPORTS) == _declared()


def test_status_strings(lib):
    assert lib.nrrs_status_string(0) == b"ok"
    assert lib.nrrs_status_string(-5).startswith(b"queue overflow")
    lib.nrrs_destroy(None)  # NULL is ignored


def test_create_rejects_bad_config(lib):
    from paper_2510_07868_amd import nrrs
    h = ctypes.c_void_p()
    bad = nrrs.Config(0, 4, 1, 2.0, 1.0, 0, 0, 4, 0, 0, 0.0, 0, 0.0)   # width 0
    assert lib.nrrs_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    bad = nrrs.Config(4, 4, 1, 2.0, 1.0, 0, 0, 9, 0, 0, 0.0, 0, 0.0)   # net_max_depth > 4
    assert lib.nrrs_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    bad = nrrs.Config(4, 4, 1, 2.0, 1.0, 0, 0, 4, 0, 0, 0.0, 7, 0.0)   # unknown loss
    assert lib.nrrs_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    bad = nrrs.Config(4, 4, 1, 2.0, 1.0, 0, 0, 4, 0, 0, 0.0, 0, 1.0)   # ema decay must be < 1
    assert lib.nrrs_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
