"""The ALU probe library (no GPU): it loads, exports its entry point and
rejects bad arguments before touching the device."""
import ctypes

import pytest


def test_probe_library_exports_and_rejects_bad_arguments():
    from paper_2303_10440_amd import probe
    if not probe.LIB_PATH.exists():
        pytest.skip("probe library not built")
    L = probe._load()
    ms = ctypes.c_double(-1.0)
    assert L.dmp_alu_time(0, 6, 16, 16, 1, ctypes.byref(ms)) == -1
    assert L.dmp_alu_time(0, 0, 0, 16, 1, ctypes.byref(ms)) == -1
    assert L.dmp_alu_time(0, 0, 16, 16, 1, None) == -1
    assert ms.value == -1.0
