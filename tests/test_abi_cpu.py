"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, and rejects bad arguments before touching a device."""
import ctypes
import re

import pytest

dm = pytest.importorskip("paper_2303_10440_amd")


def test_library_exports_every_header_symbol():
    L = dm.lib()
    names = dm.header_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n


def test_header_declares_extern_c_and_status_codes():
    text = dm.HEADER.read_text()
    assert 'extern "C"' in text
    for code in ("DM_OK", "DM_ERR_ARG", "DM_ERR_MESH", "DM_ERR_PSF", "DM_ERR_BUDGET", "DM_ERR_DEVICE"):
        assert re.search(rf"\b{code}\b", text)


def test_version_and_null_arguments():
    L = dm.lib()
    assert "gfx950" in dm.version()
    g = dm.CGrid()
    p = dm.CPsf()
    m = dm.CMesh()
    assert L.dm_render(None, ctypes.byref(m), ctypes.byref(p), ctypes.byref(g), None, None, None) == -1
    assert b"NULL" in L.dm_last_error()
    assert L.dm_render_vjp(None, None, None, None, None, None, None, None, None, None) == -1
    assert L.dm_topology_create(None, None, 0, 0, 0, None) == -1
    assert L.dm_destroy(None) == 0
    assert L.dm_topology_destroy(None) == 0
    out = ctypes.c_void_p()
    # a device index that cannot exist is refused with DM_ERR_DEVICE
    assert L.dm_create(ctypes.byref(out), 4096, 0) == -5
    assert not out.value
