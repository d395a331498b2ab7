"""FP64 reference renderer built on the C direct sums in ``meshft_oracle.c``.

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke`` and the
benchmark's CPU-baseline leg use it to check the GPU library; the library
itself never imports or calls anything here, and nothing here imports the
library.

What it computes (paper Sec. 3-4, readings listed in the design notes):

All inputs are taken as exact float64 values (callers comparing against the
float32 GPU library pass the float32-rounded values).

* frequencies: the DFT grid of an image of N_j voxels of size Delta_j,
  xi_j = 2 pi k_j / L_j with L_j = N_j Delta_j and k_j the integer DFT
  frequencies in numpy ``fftfreq`` order;
* optical transfer function of the Gaussian PSF (Eq. 2):
  h(xi) = exp(-xi^T Sigma xi / 2);
* narrow band (Sec. 5.1): frequencies where h(xi) > tau, decided as
  xi^T Sigma xi < -2 ln tau in float64 with a fixed evaluation order;
* mesh transform u(xi): the indicator transform (VOLUME) or the
  area-normalised surface transform of Eq. 5 (SURFACE);
* image (Eq. 1, product in Fourier space): I = Re(ifftn(h u 1_band)) / (Dx Dy Dz);
* gradients of a scalar loss with respect to the vertices and to the six
  covariance entries, given dL/dI, with the band held fixed.
"""
from __future__ import annotations

import ctypes
import math
import os
import pathlib
import subprocess

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
SRC = HERE / "meshft_oracle.c"
LIB = HERE / "_meshft_oracle.so"

VOLUME, SURFACE = 0, 1
# Gradient mode of mesh_ft_vjp_raw only: the unnormalised surface transform
# sum_T 2 A_T f_T (Eq. 9 summed over triangles, no 1/|Lambda|, no Eq. 6
# normalisation term).
SURFACE_RAW = 2
TWO_PI = 2.0 * np.pi


def build(force: bool = False) -> pathlib.Path:
    """Compile the C direct sums (gcc, -O2, OpenMP, no fast-math)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                        "-ffp-contract=off", "-o", str(tmp), str(SRC), "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _c():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(str(LIB))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_mesh_ft.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp, ctypes.c_int, dp]
        L.oracle_mesh_ft_vjp.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp, dp,
                                         ctypes.c_int, dp]
        L.oracle_cone_volume_ft.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp, dp, ctypes.c_int, dp]
        L.oracle_dd_exp.argtypes = [dp, ctypes.c_int, dp]
        L.oracle_tri_f.argtypes = [dp, dp]
        L.oracle_tri_dfdv.argtypes = [dp, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def num_threads() -> int:
    return int(_c().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP loops from now on (timing only; results do not
    depend on it)."""
    _c().oracle_set_num_threads(int(n))


# ---------------------------------------------------------------- primitives
def dd_exp(nodes) -> complex:
    """Divided difference of exp at up to 5 complex nodes (matrix definition)."""
    z = np.asarray(nodes, dtype=np.complex128)
    buf = _d(np.stack([z.real, z.imag], axis=1).ravel())
    out = np.zeros(2)
    _c().oracle_dd_exp(_p(buf, ctypes.c_double), len(z), _p(out, ctypes.c_double))
    return complex(out[0], out[1])


def tri_f(y) -> complex:
    """f_T of Eq. 8 from three vertex phases y_p = v_p . xi."""
    y = _d(y)
    out = np.zeros(2)
    _c().oracle_tri_f(_p(y, ctypes.c_double), _p(out, ctypes.c_double))
    return complex(out[0], out[1])


def tri_dfdv(y) -> np.ndarray:
    """Scalars B_p of Eq. 10, df_T/dv_p = xi B_p, p = 1..3."""
    y = _d(y)
    out = np.zeros(6)
    _c().oracle_tri_dfdv(_p(y, ctypes.c_double), _p(out, ctypes.c_double))
    return out[0::2] + 1j * out[1::2]


def _weights(tri_w, nt):
    if tri_w is None:
        return None, None
    w = _d(tri_w).reshape(-1)
    if w.shape[0] != nt:
        raise ValueError("one density weight per triangle")
    return w, _p(w, ctypes.c_double)


def mesh_ft_raw(V, F, xi, mode: int, tri_w=None) -> np.ndarray:
    """VOLUME: indicator transform chi(xi); SURFACE: sum_T 2 A_T f_T (unnormalised).

    ``V`` are positions relative to the phase origin, ``xi`` is [..., 3];
    ``tri_w`` (optional) are per-triangle density weights multiplying each
    triangle's term."""
    V, F = _d(V), _i(F)
    xi = _d(xi)
    shape = xi.shape[:-1]
    xi = xi.reshape(-1, 3)
    out = np.zeros(2 * xi.shape[0])
    w, wp = _weights(tri_w, F.shape[0])
    _c().oracle_mesh_ft(int(mode), _p(V, ctypes.c_double), V.shape[0], _p(F, ctypes.c_int), F.shape[0], wp,
                        _p(xi, ctypes.c_double), xi.shape[0], _p(out, ctypes.c_double))
    return (out[0::2] + 1j * out[1::2]).reshape(shape)


def cone_volume_ft(V, F, xi, c=None) -> np.ndarray:
    """Indicator transform as a sum of signed tetrahedra from the point ``c``."""
    V, F = _d(V), _i(F)
    c = _d(V.mean(axis=0) if c is None else c)
    xi = _d(xi)
    shape = xi.shape[:-1]
    xi = xi.reshape(-1, 3)
    out = np.zeros(2 * xi.shape[0])
    _c().oracle_cone_volume_ft(_p(V, ctypes.c_double), V.shape[0], _p(F, ctypes.c_int), F.shape[0],
                               _p(c, ctypes.c_double), _p(xi, ctypes.c_double), xi.shape[0],
                               _p(out, ctypes.c_double))
    return (out[0::2] + 1j * out[1::2]).reshape(shape)


def mesh_ft_vjp_raw(V, F, xi, W, mode: int, tri_w=None) -> np.ndarray:
    """Gradient with respect to V of sum_k Re[W_k u(xi_k)], where u is the
    indicator transform (VOLUME), the normalised surface transform (SURFACE)
    or the unnormalised one, sum_T 2 A_T f_T (SURFACE_RAW), all weighted by
    ``tri_w`` when given.  VOLUME and SURFACE_RAW are sums of per-triangle
    terms, so on a subset of the triangles they give those triangles' share."""
    V, F = _d(V), _i(F)
    xi = _d(xi).reshape(-1, 3)
    W = np.asarray(W, dtype=np.complex128).reshape(-1)
    Wb = _d(np.stack([W.real, W.imag], axis=1).ravel())
    dV = np.zeros((V.shape[0], 3))
    w, wp = _weights(tri_w, F.shape[0])
    _c().oracle_mesh_ft_vjp(int(mode), _p(V, ctypes.c_double), V.shape[0], _p(F, ctypes.c_int), F.shape[0], wp,
                            _p(xi, ctypes.c_double), _p(Wb, ctypes.c_double), xi.shape[0],
                            _p(dV, ctypes.c_double))
    return dV


def surface_area(V, F, tri_w=None) -> float:
    """sum_T A_T, or sum_T w_T A_T with density weights."""
    V = _d(V)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    a = 0.5 * np.linalg.norm(n, axis=1)
    return float(a.sum() if tri_w is None else (a * _d(tri_w)).sum())


def surface_area_grad(V, F, tri_w=None) -> np.ndarray:
    """d|Lambda|/dV [n_v, 3]: each triangle adds dA_T/dv_p = -w_p/2 (Sec. 4.1.2,
    w_p = e_p x N_T with e_p = v_{p-1} - v_{p+1}), times w_T if weighted;
    zero-area triangles add nothing."""
    V = _d(V)
    F = np.asarray(F, dtype=np.int64)
    P = V[F]                                   # [nt, 3 vertices, 3]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    two_a = np.linalg.norm(n, axis=1)
    N = np.divide(n, two_a[:, None], out=np.zeros_like(n), where=two_a[:, None] > 0)
    wt = np.ones(len(F)) if tri_w is None else _d(tri_w).reshape(-1)
    out = np.zeros_like(V)
    for p in range(3):
        e = P[:, (p + 2) % 3] - P[:, (p + 1) % 3]
        w = np.cross(e, N)
        np.add.at(out, F[:, p], -0.5 * w * wt[:, None])
    return out


# ---------------------------------------------------------------- frequencies
def int_freqs(n: int) -> np.ndarray:
    """Integer DFT frequencies of an n-point axis in fftfreq order."""
    return np.rint(np.fft.fftfreq(n, d=1.0 / n)).astype(np.int64)


def lengths(grid) -> np.ndarray:
    return np.array([float(grid.n[j]) * float(grid.spacing[j]) for j in range(3)])


def xi_of_k(k, grid) -> np.ndarray:
    """xi_j = (2 pi k_j) / L_j in float64; k is an integer array [..., 3]."""
    L = lengths(grid)
    k = np.asarray(k, dtype=np.float64)
    return (TWO_PI * k) / L


def quad_form(xi, sigma6) -> np.ndarray:
    """xi^T Sigma xi with Sigma = (xx, yy, zz, xy, xz, yz), in the fixed order
    ((((( Sxx x x + Syy y y) + Szz z z) + 2 Sxy x y) + 2 Sxz x z) + 2 Syz y z)."""
    s = [float(v) for v in sigma6]
    x, y, z = xi[..., 0], xi[..., 1], xi[..., 2]
    q = (s[0] * x) * x
    q = q + (s[1] * y) * y
    q = q + (s[2] * z) * z
    q = q + 2.0 * ((s[3] * x) * y)
    q = q + 2.0 * ((s[4] * x) * z)
    q = q + 2.0 * ((s[5] * y) * z)
    return q


def band_threshold(tau: float) -> float:
    """h > tau  <=>  xi^T Sigma xi < -2 ln tau  (tau = 0: everything)."""
    tau = float(tau)
    if tau <= 0.0:
        return np.inf
    return -2.0 * math.log(tau)   # the C library's log, as the band rule specifies


def full_grid_k(grid) -> np.ndarray:
    kx, ky, kz = (int_freqs(grid.n[j]) for j in range(3))
    K = np.stack(np.meshgrid(kx, ky, kz, indexing="ij"), axis=-1)
    return K


def otf_and_band(grid, sigma6, K=None):
    if K is None:
        K = full_grid_k(grid)
    xi = xi_of_k(K, grid)
    q = quad_form(xi, sigma6)
    band = q < band_threshold(grid.tau)
    h = np.exp(-0.5 * q)
    return xi, h, band


# ---------------------------------------------------------------- pipeline
def mesh_transform(V, F, xi, grid, mode: int, tri_w=None) -> np.ndarray:
    """u(xi) for positions V in the grid frame (phase origin = grid origin)."""
    Vr = _d(V) - np.asarray(grid.origin, dtype=np.float64)
    u = mesh_ft_raw(Vr, F, xi, mode, tri_w)
    if mode == SURFACE:
        u = u / surface_area(V, F, tri_w)
    return u


def spectrum(V, F, grid, sigma6, mode: int | None = None, band_sigma6=None, tri_w=None):
    """Full-grid spectrum I_hat = h u on the band (zero elsewhere).

    ``band_sigma6`` (default: ``sigma6``) selects the covariance that decides
    the band, so that derivative checks can hold the band fixed."""
    mode = grid.mode if mode is None else mode
    xi, h, band = otf_and_band(grid, sigma6)
    if band_sigma6 is not None:
        band = otf_and_band(grid, band_sigma6)[2]
    u = np.zeros(grid.n, dtype=np.complex128)
    if band.any():
        u[band] = mesh_transform(V, F, xi[band], grid, mode, tri_w)
    return h * u * band, (xi, h, band, u)


def image_of_spectrum(Ihat, grid) -> np.ndarray:
    """Re(ifftn(I_hat)) / (Dx Dy Dz) for a full-grid spectrum."""
    dvol = float(grid.spacing[0]) * float(grid.spacing[1]) * float(grid.spacing[2])
    return np.real(np.fft.ifftn(Ihat)) / dvol


def render(V, F, grid, sigma6, mode: int | None = None, band_sigma6=None, tri_w=None, return_spectrum=False):
    """Image on the grid: Re(ifftn(I_hat)) / (Dx Dy Dz).  With
    ``return_spectrum``, also the second result of ``spectrum`` (full-grid
    xi, h, band and the mesh transform u, zero off the band)."""
    Ihat, parts = spectrum(V, F, grid, sigma6, mode, band_sigma6, tri_w)
    img = image_of_spectrum(Ihat, grid)
    return (img, parts) if return_spectrum else img


def vjp_band(grid, sigma6, dL_dI):
    """The band quantities of the gradient for a given dL/dI: full-grid band
    mask, and on the band xi, h, G = fftn(dL/dI) and the adjoint weights
    W = conj(G) h / (Lx Ly Lz), so that dL/dtheta = sum_band Re[W du/dtheta]
    for the mesh transform u (band held fixed)."""
    xi, h, band = otf_and_band(grid, sigma6)
    G = np.fft.fftn(np.asarray(dL_dI, dtype=np.float64))
    LV = float(np.prod(lengths(grid)))
    xb, hb, Gb = xi[band], h[band], G[band]
    W = np.conj(Gb) * hb / LV
    return band, xb, hb, Gb, W


def psf_grad(grid, xb, hb, Gb, ub) -> np.ndarray:
    """dL/dSigma [6] from the band quantities of ``vjp_band`` and the mesh
    transform ``ub`` on the band: dh/dSigma_ab = -xi_a xi_b h / 2 (times 2 for
    an off-diagonal entry, which stands for both symmetric positions)."""
    LV = float(np.prod(lengths(grid)))
    base = np.real(np.conj(Gb) * ub * hb) / LV
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    dS = np.zeros(6)
    for i, (a, b) in enumerate(pairs):
        fac = -0.5 * xb[:, a] * xb[:, b] * (1.0 if a == b else 2.0)
        dS[i] = float(np.sum(base * fac))
    return dS


def render_vjp(V, F, grid, sigma6, dL_dI, mode: int | None = None, tri_w=None):
    """Gradients (dL/dV [n_v,3], dL/dSigma [6]) for a given dL/dI [N0,N1,N2].

    dL/dtheta = (1/(Lx Ly Lz)) sum_{k in band} Re[ conj(G_k) d(I_hat_k)/dtheta ],
    G = fftn(dL/dI), the band held fixed.  The six covariance entries are
    (xx, yy, zz, xy, xz, yz); an off-diagonal entry stands for both symmetric
    positions of Sigma."""
    mode = grid.mode if mode is None else mode
    band, xb, hb, Gb, W = vjp_band(grid, sigma6, dL_dI)
    Vr = _d(V) - np.asarray(grid.origin, dtype=np.float64)
    dV = mesh_ft_vjp_raw(Vr, F, xb, W, mode, tri_w) if band.any() else np.zeros((len(V), 3))
    u = mesh_transform(V, F, xb, grid, mode, tri_w) if band.any() else np.zeros(0, complex)
    return dV, psf_grad(grid, xb, hb, Gb, u)


# ------------------------------------------------------- tabulated OTF
def otf_band(otf, tau) -> np.ndarray:
    """Band of a tabulated OTF: Re^2 + Im^2 > tau^2 in float64."""
    otf = np.asarray(otf, dtype=np.complex128)
    re, im = otf.real, otf.imag
    return (re * re + im * im) > float(tau) * float(tau)


def render_otf(V, F, grid, otf, mode: int | None = None, tri_w=None) -> np.ndarray:
    """Image for a PSF given by its transform on the full DFT grid (an array
    of the grid's shape, numpy fftn order; Hermitian for a real PSF), the
    band being where |OTF| > tau, decided as Re^2 + Im^2 > tau^2 in float64:
    I = Re(ifftn(OTF u 1_band)) / (Dx Dy Dz)."""
    mode = grid.mode if mode is None else mode
    otf = np.asarray(otf, dtype=np.complex128)
    K = full_grid_k(grid)
    xi = xi_of_k(K, grid)
    band = otf_band(otf, grid.tau)
    u = np.zeros(grid.n, dtype=np.complex128)
    if band.any():
        u[band] = mesh_transform(V, F, xi[band], grid, mode, tri_w)
    dvol = float(grid.spacing[0]) * float(grid.spacing[1]) * float(grid.spacing[2])
    return np.real(np.fft.ifftn(otf * u * band)) / dvol


def render_otf_vjp(V, F, grid, otf, dL_dI, mode: int | None = None, tri_w=None) -> np.ndarray:
    """dL/dV for the tabulated-OTF image, given dL/dI (band held fixed):
    dL/dV = (1/(Lx Ly Lz)) sum_{k in band} Re[conj(G_k) OTF_k du_k/dV]."""
    mode = grid.mode if mode is None else mode
    otf = np.asarray(otf, dtype=np.complex128)
    K = full_grid_k(grid)
    xi = xi_of_k(K, grid)
    band = otf_band(otf, grid.tau)
    G = np.fft.fftn(np.asarray(dL_dI, dtype=np.float64))
    LV = float(np.prod(lengths(grid)))
    W = np.conj(G[band]) * otf[band] / LV
    Vr = _d(V) - np.asarray(grid.origin, dtype=np.float64)
    return mesh_ft_vjp_raw(Vr, F, xi[band], W, mode, tri_w) if band.any() else np.zeros((len(V), 3))
