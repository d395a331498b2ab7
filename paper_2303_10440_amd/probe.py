"""Vector-ALU throughput of the device (``libdmprobe.so``, include/dm_probe.h).

The sweeps are priced against the FP32 vector ALU: fused multiply-adds and
the transcendental instructions of the phase factors and reciprocals.  This
module times long independent chains of each kind and returns lane
instructions per second, so that a transcendental can be counted at its
measured cost instead of an assumed one.
"""
from __future__ import annotations

import ctypes
import pathlib

LIB_PATH = pathlib.Path(__file__).resolve().parent / "libdmprobe.so"
KINDS = {"fma": 0, "sin": 1, "cos": 2, "rcp": 3, "mix": 4, "fma_sgpr": 5}
THREADS = 256
CHAINS = 8
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2303_10440_amd/csrc/build.sh")
        import torch  # noqa: F401  (one HIP runtime in the process: torch's)
        L = ctypes.CDLL(str(LIB_PATH))
        L.dmp_alu_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double)]
        L.dmp_alu_time.restype = ctypes.c_int
        _lib = L
    return _lib


def alu_time_ms(kind: str, blocks: int, iters: int, reps: int = 5, device: int = 0) -> float:
    ms = ctypes.c_double()
    rc = _load().dmp_alu_time(device, KINDS[kind], blocks, iters, reps, ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"dmp_alu_time({kind}) failed with status {rc}")
    return ms.value


def alu_rates(device: int = 0, blocks: int = 2048, iters: int = 4096) -> dict:
    """Lane instructions per second of each kind ("fma": all operands in
    VGPRs; "fma_sgpr": one operand in an SGPR), and how the mixed stream
    (8 FMA and 2 sine chains per step) compares with the two kinds' times
    added (1.0: no overlap; max/sum: full overlap)."""
    lanes = blocks * THREADS * iters
    out = {}
    for kind in ("fma", "fma_sgpr", "sin", "cos", "rcp"):
        out[kind] = lanes * CHAINS / (alu_time_ms(kind, blocks, iters, device=device) * 1e-3)
    t_mix = alu_time_ms("mix", blocks, iters, device=device) * 1e-3
    t_fma, t_sin = lanes * CHAINS / out["fma"], lanes * 2 / out["sin"]
    out["mix_over_sum"] = t_mix / (t_fma + t_sin)
    out["max_over_sum"] = max(t_fma, t_sin) / (t_fma + t_sin)
    out["config"] = f"{blocks} workgroups x {THREADS} lanes x {iters} steps x {CHAINS} chains"
    return out
