"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/tp.h is exported by libtp.so, and argument errors are reported before
anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(tp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1806_07247_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtp.so not built")
    return _lib.load()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("tp_tprod",):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_1806_07247_amd", "libtp.so"))
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(lib):
    from paper_1806_07247_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def test_tprod_argument_errors(lib):
    ws = lib.tp_tprod_workspace_size(4, 3, 2, 5, 0)
    assert ws > 0
    assert lib.tp_tprod(None, FAKE, FAKE, 4, 3, 2, 5, 0, FAKE, ws, None) == -1
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 5, 7, FAKE, ws, None) == -1
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 0, 3, 2, 5, 0, FAKE, ws, None) == -2
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 0, 0, FAKE, ws, None) == -2
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 2000, 0, FAKE, ws, None) == -2
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 5, 0, FAKE, ws - 1, None) == -3
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 5, 0, None, ws, None) == -3
    assert lib.tp_status_string(-3) == b"workspace missing or too small"


def test_workspace_query(lib):
    # half spectra of A, B, C: 2 planes * (n3/2+1) slices each, 256-byte aligned
    h = 5 // 2 + 1
    need = sum(((2 * h * e * 4 + 255) // 256) * 256 for e in (4 * 3, 3 * 2, 4 * 2))
    assert lib.tp_tprod_workspace_size(4, 3, 2, 5, 0) >= need
    assert lib.tp_tprod_workspace_size(0, 3, 2, 5, 0) == 0
