"""The C-ABI library builds, loads and exports every symbol include/retina.h
declares; host-side argument checks that need no GPU."""
import ctypes
import os
import re

import pytest

from paper_1709_08610_amd import retina

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "retina.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(retina_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(retina.LIB_PATH):
        from paper_1709_08610_amd import build
        build.build()
    return retina.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("retina_create", "retina_destroy", "retina_last_error", "retina_response",
              "retina_find_tracks"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(retina.EXPORTS) == sorted(_declared())


def test_struct_sizes_match_header():
    # retina_track is documented as 48 bytes; the binding's layout must agree
    assert ctypes.sizeof(retina.Track) == 48
    assert ctypes.sizeof(retina.Hits) == 48
    assert ctypes.sizeof(retina.Geometry) == 16


def test_null_context_paths(lib):
    assert lib.retina_last_error(None) == b"retina: NULL context"
    assert lib.retina_response(None, None, None, None, 0, None, 1.0, 1, None, None, None) == retina.ERR_INVALID_ARG
    assert lib.retina_find_tracks(None, None, None, None, None, 0, None, None, None) == retina.ERR_INVALID_ARG
    assert lib.retina_set_stream(None, None) == retina.ERR_INVALID_ARG
    lib.retina_destroy(None)  # NULL-safe


def test_create_without_gfx950_device(lib):
    """Here (no GPU) retina_create must fail cleanly with RETINA_ERR_DEVICE."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p(123)
    assert lib.retina_create(0, ctypes.byref(h)) == retina.ERR_DEVICE
    assert not h.value
    with pytest.raises(retina.RetinaError):
        retina.Context(0)
