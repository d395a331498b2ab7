"""Python binding of libdeltamic (the gfx950 mesh-transform microscope renderer).

Argument marshalling only: every step of the render and of its gradient runs
in the HIP kernels behind the C ABI of ``include/deltamic.h``.  PyTorch is
used for device memory and streams.  There is no CPU fallback: if the
library is missing or no gfx950 device is present, calls raise.

Typical use::

    import paper_2303_10440_amd as dm
    h = dm.Handle(device=0)
    topo = h.topology(faces)                     # int32 [n_t, 3], validated once
    img = dm.render(h, verts, topo, sigma6, grid)  # verts: float32 cuda [n_v, 3]

    # differentiable:
    img = dm.RenderFunction.apply(verts, sigma6_tensor, h, topo, grid)
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import re

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
LIB_PATH = HERE / "libdeltamic.so"
HEADER = HERE.parent / "include" / "deltamic.h"

VOLUME, SURFACE = 0, 1
STATUS = {0: "DM_OK", -1: "DM_ERR_ARG", -2: "DM_ERR_MESH", -3: "DM_ERR_PSF", -4: "DM_ERR_BUDGET",
          -5: "DM_ERR_DEVICE", -6: "DM_ERR_FFT", -7: "DM_ERR_BUSY", -8: "DM_ERR_STATE"}


class DeltamicError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} failed with {STATUS.get(status, status)}: {msg}")
        self.status = status


class CGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("spacing", ctypes.c_float * 3), ("origin", ctypes.c_float * 3),
                ("band_tau", ctypes.c_float), ("mode", ctypes.c_int32)]


class CPsf(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_float * 6)]


class CKernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("pairs", ctypes.c_double)]


class CMesh(ctypes.Structure):
    _fields_ = [("verts_dev", ctypes.c_void_p), ("n_verts", ctypes.c_int32), ("topo", ctypes.c_void_p)]


class CServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_size_t)]


class CServeRequest(ctypes.Structure):
    _fields_ = [("mesh_id", ctypes.c_int32), ("psf", CPsf), ("grid", CGrid), ("dL_dimage_dev", ctypes.c_void_p),
                ("image_dev", ctypes.c_void_p), ("dL_dverts_dev", ctypes.c_void_p), ("dL_dsigma_dev", ctypes.c_void_p),
                ("otf_dev", ctypes.c_void_p)]


class CServeResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("batch_size", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class CServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("mean_batch", ctypes.c_double), ("peak_inflight_bytes", ctypes.c_size_t)]


class CRequest(ctypes.Structure):
    _fields_ = [("mesh", CMesh), ("psf", CPsf), ("grid", CGrid), ("dL_dimage_dev", ctypes.c_void_p),
                ("image_dev", ctypes.c_void_p), ("dL_dverts_dev", ctypes.c_void_p), ("dL_dsigma_dev", ctypes.c_void_p),
                ("otf_dev", ctypes.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2303_10440_amd/csrc/build.sh "
                          "(or __graft_entry__.build())")
    # torch ships its own HIP runtime.  Loading torch first makes the library bind
    # to that same runtime (matched by soname); loading the library first would
    # bring in a second HIP/HSA runtime under which torch finds no GPU.
    import torch  # noqa: F401
    L = ctypes.CDLL(str(LIB_PATH))
    vp, i32, i64, fp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_float)
    sig = {
        "dm_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t],
        "dm_destroy": [vp],
        "dm_memory_in_use": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "dm_topology_create": [vp, vp, i32, i32, ctypes.c_int, ctypes.POINTER(vp)],
        "dm_topology_destroy": [vp],
        "dm_topology_info": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "dm_topology_strips": [vp, i32, vp, vp, ctypes.POINTER(i32)],
        "dm_laplace_smooth": [vp, vp, ctypes.c_float, vp, vp, i32, ctypes.c_float, vp, vp],
        "dm_topology_set_weights": [vp, vp],
        "dm_render_otf": [vp, ctypes.POINTER(CMesh), vp, ctypes.POINTER(CGrid), vp, vp],
        "dm_render_otf_vjp": [vp, ctypes.POINTER(CMesh), vp, ctypes.POINTER(CGrid), vp, vp, vp, vp],
        "dm_band_size": [vp, ctypes.POINTER(CGrid), ctypes.POINTER(CPsf), ctypes.POINTER(i64), vp],
        "dm_band_export": [vp, ctypes.POINTER(CGrid), ctypes.POINTER(CPsf), vp, vp, vp, vp],
        "dm_render": [vp, ctypes.POINTER(CMesh), ctypes.POINTER(CPsf), ctypes.POINTER(CGrid), vp, vp, vp],
        "dm_render_vjp": [vp, ctypes.POINTER(CMesh), ctypes.POINTER(CPsf), ctypes.POINTER(CGrid), vp, vp, vp, vp,
                          vp, vp],
        "dm_mesh_transform": [vp, ctypes.POINTER(CMesh), ctypes.POINTER(CGrid), vp, i64, vp, vp],
        "dm_mesh_transform_noalloc": [vp, ctypes.POINTER(CMesh), ctypes.POINTER(CGrid), vp, i64, vp, vp],
        "dm_timing_enable": [vp, ctypes.c_int],
        "dm_timing_read": [vp, ctypes.POINTER(CKernelTime), ctypes.POINTER(CKernelTime), ctypes.POINTER(CKernelTime),
                           ctypes.POINTER(CKernelTime), ctypes.c_int],
        "dm_batch_run": [vp, i32, vp, vp],
        "dm_server_create": [ctypes.c_int, ctypes.POINTER(CServerConfig), ctypes.POINTER(vp)],
        "dm_server_destroy": [vp],
        "dm_server_mesh_add": [vp, vp, i32, vp, i32, ctypes.POINTER(i32)],
        "dm_server_mesh_remove": [vp, i32],
        "dm_submit": [vp, ctypes.POINTER(CServeRequest), ctypes.POINTER(ctypes.c_uint64)],
        "dm_poll": [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(CServeResult)],
        "dm_server_stats_read": [vp, ctypes.POINTER(CServerStats)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.dm_last_error.restype = ctypes.c_char_p
    L.dm_last_error.argtypes = []
    L.dm_version.restype = ctypes.c_char_p
    L.dm_version.argtypes = []
    _lib = L
    return L


def lib():
    return _load()


def header_symbols() -> list[str]:
    """Entry points declared in include/deltamic.h."""
    text = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:dm_status|const char\*)\s+(dm_\w+)\s*\(", text, flags=re.M)))


def _check(status: int, func: str):
    if status != 0:
        raise DeltamicError(status, func, _load().dm_last_error().decode())


def version() -> str:
    return _load().dm_version().decode()


# ------------------------------------------------------------------ helpers
def _grid(g) -> CGrid:
    c = CGrid()
    for j in range(3):
        c.n[j] = int(g.n[j])
        c.spacing[j] = float(g.spacing[j])
        c.origin[j] = float(g.origin[j])
    c.band_tau = float(g.tau)
    c.mode = int(g.mode)
    return c


def _psf(sigma6) -> CPsf:
    p = CPsf()
    vals = sigma6.detach().cpu().tolist() if hasattr(sigma6, "detach") else list(sigma6)
    if len(vals) != 6:
        raise ValueError("sigma must have 6 entries (xx, yy, zz, xy, xz, yz)")
    for j in range(6):
        p.sigma[j] = float(vals[j])
    return p


def _torch():
    import torch
    return torch


def _stream(device: int):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(x, dtype, shape_last=None, name="tensor"):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if shape_last is not None and (x.dim() != 2 or x.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape [n, {shape_last}]")
    return x.contiguous()


class Handle:
    """Owns a dm_handle on one device (workspace, band cache, FFT plans)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        L = _load()
        self.device = int(device)
        self._h = ctypes.c_void_p()
        _check(L.dm_create(ctypes.byref(self._h), self.device, ctypes.c_size_t(int(hbm_budget_bytes))), "dm_create")

    @property
    def ptr(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _load().dm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def memory_in_use(self) -> int:
        v = ctypes.c_size_t()
        _check(_load().dm_memory_in_use(self._h, ctypes.byref(v)), "dm_memory_in_use")
        return int(v.value)

    def timing(self, enable: bool):
        _check(_load().dm_timing_enable(self._h, 1 if enable else 0), "dm_timing_enable")

    def timing_read(self, reset: bool = True) -> dict:
        """{'fwd': (launches, ms, pairs), 'vjp': ..., 'batch': ..., 'fused': ...}
        from the HIP events the library records around each sweep launch."""
        a, b, c, d = CKernelTime(), CKernelTime(), CKernelTime(), CKernelTime()
        _check(_load().dm_timing_read(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                      1 if reset else 0), "dm_timing_read")
        return {"fwd": (int(a.launches), float(a.ms), float(a.pairs)),
                "vjp": (int(b.launches), float(b.ms), float(b.pairs)),
                "batch": (int(c.launches), float(c.ms), float(c.pairs)),
                "fused": (int(d.launches), float(d.ms), float(d.pairs))}

    def topology(self, faces, n_verts: int | None = None) -> "Topology":
        return Topology(self, faces, n_verts)


class Topology:
    """Validated faces + vertex incidence of one mesh (dm_topology)."""

    def __init__(self, handle: Handle, faces, n_verts: int | None = None):
        L = _load()
        self.handle = handle
        torch = _torch()
        if isinstance(faces, torch.Tensor):
            f = faces.detach().to(torch.int32).contiguous()
            on_dev = 1 if f.is_cuda else 0
            arr = f
            ptr = f.data_ptr()
            nf = f.shape[0]
            nv = int(n_verts) if n_verts is not None else (int(f.max().item()) + 1 if nf else 0)
        else:
            arr = np.ascontiguousarray(np.asarray(faces, dtype=np.int32))
            on_dev = 0
            ptr = arr.ctypes.data
            nf = arr.shape[0]
            nv = int(n_verts) if n_verts is not None else (int(arr.max()) + 1 if nf else 0)
        if arr.ndim != 2 or arr.shape[1] != 3:
            raise ValueError("faces must have shape [n_t, 3]")
        self._t = ctypes.c_void_p()
        _check(L.dm_topology_create(handle.ptr, ctypes.c_void_p(ptr), int(nf), int(nv), on_dev, ctypes.byref(self._t)),
               "dm_topology_create")
        self.n_faces, self.n_verts = int(nf), int(nv)
        c = ctypes.c_int32()
        _check(L.dm_topology_info(self._t, None, None, ctypes.byref(c)), "dm_topology_info")
        self.closed = bool(c.value)

    def set_weights(self, weights=None):
        """Per-face density weights (input face order) or None for all 1;
        updates ``closed`` (weighted closure for the indicator density)."""
        L = _load()
        if weights is None:
            _check(L.dm_topology_set_weights(self._t, None), "dm_topology_set_weights")
        else:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).reshape(-1))
            if w.shape[0] != self.n_faces:
                raise ValueError(f"need {self.n_faces} weights")
            _check(L.dm_topology_set_weights(self._t, ctypes.c_void_p(w.ctypes.data)), "dm_topology_set_weights")
        c = ctypes.c_int32()
        _check(L.dm_topology_info(self._t, None, None, ctypes.byref(c)), "dm_topology_info")
        self.closed = bool(c.value)

    @property
    def ptr(self):
        return self._t

    def close(self):
        if getattr(self, "_t", None) and self._t.value:
            _load().dm_topology_destroy(self._t)
            self._t = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def laplace_smooth(h: Handle, topo: Topology, grad, lam: float = 50.0, max_iter: int = 2000, tol: float = 1e-6,
                   out=None, with_info: bool = False):
    """(I + lam L)^{-2} grad on the device (dm_laplace_smooth); grad is a
    float32 [n_verts, 3] device tensor.  With with_info, also returns
    (iterations, relative residual) of both solves."""
    torch = _torch()
    if not (isinstance(grad, torch.Tensor) and grad.is_cuda and grad.dtype == torch.float32):
        raise TypeError("grad must be a float32 device tensor")
    if tuple(grad.shape) != (topo.n_verts, 3):
        raise ValueError(f"grad must have shape [{topo.n_verts}, 3]")
    g = grad.contiguous()
    if out is None:
        out = torch.empty_like(g)
    info = torch.zeros(4, dtype=torch.float32, device=g.device) if with_info else None
    _check(_load().dm_laplace_smooth(h.ptr, topo.ptr, float(lam), ctypes.c_void_p(g.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), int(max_iter), float(tol),
                                     ctypes.c_void_p(info.data_ptr() if info is not None else 0),
                                     _stream(g.device.index or 0)), "dm_laplace_smooth")
    if with_info:
        i = info.cpu().tolist()
        return out, {"iters": (int(i[0]), int(i[2])), "residual": (i[1], i[3])}
    return out


def _mesh(verts, topo: Topology) -> CMesh:
    m = CMesh()
    m.verts_dev = ctypes.c_void_p(verts.data_ptr())
    m.n_verts = int(verts.shape[0])
    m.topo = topo.ptr
    return m


# ----------------------------------------------------------------- calls
def topology_strips(faces):
    """The strip order a topology uses (host only): (faces [n,3] int32 in strip
    order, flags [n] int32 (bit 0 strip start, bit 1 reversed orientation),
    number of strips)."""
    F = np.ascontiguousarray(np.asarray(faces, dtype=np.int32).reshape(-1, 3))
    out = np.zeros_like(F)
    flags = np.zeros(len(F), np.int32)
    ns = ctypes.c_int32()
    _check(_load().dm_topology_strips(ctypes.c_void_p(F.ctypes.data), len(F), ctypes.c_void_p(out.ctypes.data),
                                      ctypes.c_void_p(flags.ctypes.data), ctypes.byref(ns)), "dm_topology_strips")
    return out, flags, int(ns.value)


def band_size(h: Handle, grid, sigma6) -> int:
    n = ctypes.c_int64()
    g, p = _grid(grid), _psf(sigma6)
    _check(_load().dm_band_size(h.ptr, ctypes.byref(g), ctypes.byref(p), ctypes.byref(n), _stream(h.device)),
           "dm_band_size")
    return int(n.value)


def band_export(h: Handle, grid, sigma6) -> dict:
    n = band_size(h, grid, sigma6)
    k = np.zeros((n, 3), np.int32)
    pos = np.zeros(n, np.int64)
    w = np.zeros(n, np.float32)
    g, p = _grid(grid), _psf(sigma6)
    _check(_load().dm_band_export(h.ptr, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(k.ctypes.data),
                                  ctypes.c_void_p(pos.ctypes.data), ctypes.c_void_p(w.ctypes.data),
                                  _stream(h.device)), "dm_band_export")
    return {"k": k, "pos": pos, "weight": w}


def render(h: Handle, verts, topo: Topology, sigma6, grid, spectrum: bool = False):
    """Image [n0, n1, n2] float32 (and the band spectrum [n_entries, 2] if asked)."""
    torch = _torch()
    verts = _dev_tensor(verts, torch.float32, 3, "verts")
    g, p, m = _grid(grid), _psf(sigma6), _mesh(verts, topo)
    img = torch.empty(tuple(int(x) for x in grid.n), dtype=torch.float32, device=verts.device)
    spec = None
    if spectrum:
        spec = torch.empty((band_size(h, grid, sigma6), 2), dtype=torch.float32, device=verts.device)
    _check(_load().dm_render(h.ptr, ctypes.byref(m), ctypes.byref(p), ctypes.byref(g), ctypes.c_void_p(img.data_ptr()),
                             ctypes.c_void_p(spec.data_ptr() if spec is not None else 0), _stream(h.device)),
           "dm_render")
    return (img, spec) if spectrum else img


def render_vjp(h: Handle, verts, topo: Topology, sigma6, grid, dL_dimage, want_verts: bool = True,
               want_sigma: bool = True, want_image: bool = False, spectrum_in=None):
    """(dL/dverts [n_v,3] | None, dL/dsigma [6] | None, image | None)."""
    torch = _torch()
    verts = _dev_tensor(verts, torch.float32, 3, "verts")
    gI = _dev_tensor(dL_dimage, torch.float32, None, "dL_dimage")
    if tuple(gI.shape) != tuple(int(x) for x in grid.n):
        raise ValueError("dL_dimage must have the grid's shape")
    g, p, m = _grid(grid), _psf(sigma6), _mesh(verts, topo)
    dv = torch.empty_like(verts) if want_verts else None
    ds = torch.empty(6, dtype=torch.float32, device=verts.device) if want_sigma else None
    img = torch.empty(tuple(int(x) for x in grid.n), dtype=torch.float32, device=verts.device) if want_image else None
    sp = None
    if spectrum_in is not None:
        sp = _dev_tensor(spectrum_in, torch.float32, 2, "spectrum_in")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
    _check(_load().dm_render_vjp(h.ptr, ctypes.byref(m), ctypes.byref(p), ctypes.byref(g), ptr(gI), ptr(dv), ptr(ds),
                                 ptr(img), ptr(sp), _stream(h.device)), "dm_render_vjp")
    return dv, ds, img


def _otf_tensor(otf, grid):
    torch = _torch()
    n0, n1, n2 = (int(x) for x in grid.n)
    if not (isinstance(otf, torch.Tensor) and otf.is_cuda and otf.dtype == torch.complex64):
        raise TypeError("otf must be a complex64 device tensor")
    if tuple(otf.shape) != (n0, n1, n2 // 2 + 1):
        raise ValueError(f"otf must have shape ({n0}, {n1}, {n2 // 2 + 1}) (half spectrum)")
    return otf.contiguous()


def render_otf(h: Handle, verts, topo: Topology, otf, grid):
    """Image for a tabulated PSF (dm_render_otf): ``otf`` is the complex64
    half spectrum [n0, n1, n2 // 2 + 1] of the PSF's transform."""
    torch = _torch()
    verts = _dev_tensor(verts, torch.float32, 3, "verts")
    o = _otf_tensor(otf, grid)
    g, m = _grid(grid), _mesh(verts, topo)
    img = torch.empty(tuple(int(x) for x in grid.n), dtype=torch.float32, device=verts.device)
    _check(_load().dm_render_otf(h.ptr, ctypes.byref(m), ctypes.c_void_p(o.data_ptr()), ctypes.byref(g),
                                 ctypes.c_void_p(img.data_ptr()), _stream(h.device)), "dm_render_otf")
    return img


def render_otf_vjp(h: Handle, verts, topo: Topology, otf, grid, dL_dimage, want_image: bool = False):
    """(dL/dverts, image | None) for a tabulated PSF (dm_render_otf_vjp)."""
    torch = _torch()
    verts = _dev_tensor(verts, torch.float32, 3, "verts")
    o = _otf_tensor(otf, grid)
    gI = _dev_tensor(dL_dimage, torch.float32, None, "dL_dimage")
    if tuple(gI.shape) != tuple(int(x) for x in grid.n):
        raise ValueError("dL_dimage must have the grid's shape")
    g, m = _grid(grid), _mesh(verts, topo)
    dv = torch.empty_like(verts)
    img = torch.empty(tuple(int(x) for x in grid.n), dtype=torch.float32, device=verts.device) if want_image else None
    _check(_load().dm_render_otf_vjp(h.ptr, ctypes.byref(m), ctypes.c_void_p(o.data_ptr()), ctypes.byref(g),
                                     ctypes.c_void_p(gI.data_ptr()), ctypes.c_void_p(dv.data_ptr()),
                                     ctypes.c_void_p(img.data_ptr() if img is not None else 0), _stream(h.device)),
           "dm_render_otf_vjp")
    return dv, img


def batch_run(h: Handle, requests, want_image: bool = True, want_verts: bool = True, want_sigma: bool = True):
    """Runs many independent requests as one batch (dm_batch_run).

    ``requests``: sequence of (verts, topo, sigma6, grid, dL_dimage or None)
    or (verts, topo, sigma6, grid, dL_dimage or None, otf): with a tabulated
    OTF (complex64 half spectrum, as in render_otf) sigma6 is ignored (may be
    None) and the request has no dL/dsigma.
    Returns a list of (image | None, dL/dverts | None, dL/dsigma | None)."""
    torch = _torch()
    n = len(requests)
    arr = (CRequest * max(n, 1))()
    outs, keep = [], []
    for i, req in enumerate(requests):
        if len(req) not in (5, 6):
            raise ValueError("a request is (verts, topo, sigma6, grid, dL_dimage[, otf])")
        verts, topo, sigma6, grid, gI = req[:5]
        otf = req[5] if len(req) == 6 else None
        otf = _otf_tensor(otf, grid) if otf is not None else None
        verts = _dev_tensor(verts, torch.float32, 3, "verts")
        shape = tuple(int(x) for x in grid.n)
        if gI is not None:
            gI = _dev_tensor(gI, torch.float32, None, "dL_dimage")
            if tuple(gI.shape) != shape:
                raise ValueError("dL_dimage must have the grid's shape")
        img = torch.empty(shape, dtype=torch.float32, device=verts.device) if want_image else None
        dv = torch.empty_like(verts) if (want_verts and gI is not None) else None
        ds = (torch.empty(6, dtype=torch.float32, device=verts.device)
              if (want_sigma and gI is not None and otf is None) else None)
        r = arr[i]
        r.mesh = _mesh(verts, topo)
        r.psf = _psf(sigma6) if otf is None else CPsf()
        r.otf_dev = otf.data_ptr() if otf is not None else None
        r.grid = _grid(grid)
        r.dL_dimage_dev = gI.data_ptr() if gI is not None else None
        r.image_dev = img.data_ptr() if img is not None else None
        r.dL_dverts_dev = dv.data_ptr() if dv is not None else None
        r.dL_dsigma_dev = ds.data_ptr() if ds is not None else None
        outs.append((img, dv, ds))
        keep.append((verts, gI, otf))
    _check(_load().dm_batch_run(h.ptr, n, ctypes.cast(arr, ctypes.c_void_p), _stream(h.device)), "dm_batch_run")
    return outs


class Server:
    """Continuous-batching server (dm_server_*): resident meshes, submit/poll."""

    def __init__(self, device: int = 0, max_batch: int = 32, max_inflight: int = 2, queue_capacity: int = 100000,
                 hbm_budget_bytes: int = 0):
        L = _load()
        cfg = CServerConfig(int(max_batch), int(max_inflight), int(queue_capacity), int(hbm_budget_bytes))
        self.device = int(device)
        self._s = ctypes.c_void_p()
        _check(L.dm_server_create(self.device, ctypes.byref(cfg), ctypes.byref(self._s)), "dm_server_create")

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            _load().dm_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mesh_add(self, V, F) -> int:
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float32))
        F = np.ascontiguousarray(np.asarray(F, dtype=np.int32))
        mid = ctypes.c_int32()
        _check(_load().dm_server_mesh_add(self._s, ctypes.c_void_p(V.ctypes.data), V.shape[0],
                                          ctypes.c_void_p(F.ctypes.data), F.shape[0], ctypes.byref(mid)),
               "dm_server_mesh_add")
        return int(mid.value)

    def mesh_remove(self, mesh_id: int):
        _check(_load().dm_server_mesh_remove(self._s, int(mesh_id)), "dm_server_mesh_remove")

    def submit(self, mesh_id: int, sigma6, grid, dL_dimage=None, image=None, dverts=None, dsigma=None,
               otf=None) -> int:
        """Queues a request; the tensors must stay alive until poll() reports it.
        ``otf``: a tabulated OTF (complex64 half spectrum on the device, as in
        render_otf) instead of sigma6 (then ignored; no dsigma)."""
        r = CServeRequest()
        r.mesh_id = int(mesh_id)
        r.psf = _psf(sigma6) if otf is None else CPsf()
        r.grid = _grid(grid)
        p = lambda t: t.data_ptr() if t is not None else None
        r.dL_dimage_dev, r.image_dev, r.dL_dverts_dev, r.dL_dsigma_dev = p(dL_dimage), p(image), p(dverts), p(dsigma)
        if otf is not None:
            o = _otf_tensor(otf, grid)
            if o is not otf:
                raise ValueError("otf must be contiguous (the server reads it when the request runs)")
            r.otf_dev = o.data_ptr()
        t = ctypes.c_uint64()
        _check(_load().dm_submit(self._s, ctypes.byref(r), ctypes.byref(t)), "dm_submit")
        return int(t.value)

    def poll(self, ticket: int, blocking: bool = True):
        """None while pending; else {'status', 'batch_size', 'queue_ms', 'total_ms'}."""
        res = CServeResult()
        st = _load().dm_poll(self._s, ctypes.c_uint64(ticket), 1 if blocking else 0, ctypes.byref(res))
        if st == -7:
            return None
        _check(st, "dm_poll")
        return {"status": int(res.status), "batch_size": int(res.batch_size), "queue_ms": float(res.queue_ms),
                "total_ms": float(res.total_ms)}

    def stats(self) -> dict:
        st = CServerStats()
        _check(_load().dm_server_stats_read(self._s, ctypes.byref(st)), "dm_server_stats_read")
        return {k: getattr(st, k) for k, _ in CServerStats._fields_}


def mesh_transform(h: Handle, verts, topo: Topology, grid, k, out=None, noalloc: bool = False):
    """u_hat(2 pi k / L) as complex64 [n] for integer frequencies k [n, 3].

    out: optional float32 [n, 2] device tensor to write into.  noalloc: call
    dm_mesh_transform_noalloc, which works in the library's fixed scratch and
    allocates nothing (pass `out` and a device int32 `k` to keep the whole
    call allocation-free)."""
    torch = _torch()
    verts = _dev_tensor(verts, torch.float32, 3, "verts")
    if not isinstance(k, torch.Tensor):
        k = torch.as_tensor(np.asarray(k, dtype=np.int32))
    k = k.to(device=verts.device, dtype=torch.int32).contiguous()
    if out is None:
        out = torch.empty((k.shape[0], 2), dtype=torch.float32, device=verts.device)
    elif tuple(out.shape) != (k.shape[0], 2) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of shape [n, 2]")
    g, m = _grid(grid), _mesh(verts, topo)
    name = "dm_mesh_transform_noalloc" if noalloc else "dm_mesh_transform"
    _check(getattr(_load(), name)(h.ptr, ctypes.byref(m), ctypes.byref(g), ctypes.c_void_p(k.data_ptr()),
                                  int(k.shape[0]), ctypes.c_void_p(out.data_ptr()), _stream(h.device)), name)
    return torch.view_as_complex(out)


def _autograd_function():
    torch = _torch()

    class RenderFunction(torch.autograd.Function):
        """image = render(verts, sigma6); backward gives dL/dverts and dL/dsigma6.

        sigma6 is a 6-vector tensor (xx, yy, zz, xy, xz, yz); its values are
        read on the host (the band depends on them).  The forward saves the
        band spectrum so the backward skips the forward sweep."""

        @staticmethod
        def forward(ctx, verts, sigma6, handle, topo, grid):
            img, spec = render(handle, verts, topo, sigma6, grid, spectrum=True)
            ctx.save_for_backward(verts, sigma6, spec)
            ctx.handle, ctx.topo, ctx.grid = handle, topo, grid
            return img

        @staticmethod
        def backward(ctx, grad):
            verts, sigma6, spec = ctx.saved_tensors
            dv, ds, _ = render_vjp(ctx.handle, verts, ctx.topo, sigma6, ctx.grid, grad.contiguous(),
                                   want_verts=ctx.needs_input_grad[0], want_sigma=ctx.needs_input_grad[1],
                                   spectrum_in=spec)
            if ds is not None:
                ds = ds.to(sigma6.dtype).to(sigma6.device)
            return dv, ds, None, None, None

    return RenderFunction


class _Lazy:
    _cls = None

    def __get__(self, obj, owner):
        if _Lazy._cls is None:
            _Lazy._cls = _autograd_function()
        return _Lazy._cls


class _NS:
    RenderFunction = _Lazy()


def __getattr__(name):
    if name == "RenderFunction":
        return _NS.RenderFunction
    raise AttributeError(name)


_load()
