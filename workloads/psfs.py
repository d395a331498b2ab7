"""Seeded tabulated optical transfer functions: stand-ins for measured or
physics-based PSFs given as arrays (the paper's Sec. 3.2 and conclusion name
experimental and aberrated PSFs as the step beyond its Gaussian).

This module builds inputs only.  A table is an array of the grid's shape in
numpy fftn order (or its half spectrum, kz in [0, n2/2]), Hermitian, so that
it is the transform of a real PSF: an even, decaying envelope, an odd phase
(defocus-like aberration) and an even support mask (a widefield-like missing
cone).  Positions on the Nyquist planes of even axes are set to zero, which
keeps the table exactly Hermitian there.
"""
from __future__ import annotations

import numpy as np


def _freqs(grid):
    n = [int(x) for x in grid.n]
    L = [n[j] * float(grid.spacing[j]) for j in range(3)]
    k = [np.rint(np.fft.fftfreq(n[j], d=1.0 / n[j])) for j in range(3)]
    X, Y, Z = np.meshgrid(*[2.0 * np.pi * k[j] / L[j] for j in range(3)], indexing="ij")
    nyq = np.zeros(n, dtype=bool)
    for j, A in enumerate(np.meshgrid(*k, indexing="ij")):
        if n[j] % 2 == 0:
            nyq |= A == -(n[j] // 2)
    return X, Y, Z, nyq


def aberrated_otf(grid, width_xy: float, width_z: float, defocus: float = 0.0, cone: float | None = None,
                  half: bool = False) -> np.ndarray:
    """(1 + (xi_x^2 + xi_y^2) w_xy^2 + xi_z^2 w_z^2)^-2  *  exp(i defocus (xi_x^2 + xi_y^2) xi_z w_xy^2 w_z)
    * [|xi_z| w_z <= cone * sqrt(xi_x^2 + xi_y^2) w_xy + 1]  (the mask only if ``cone`` is given);
    complex64, zero on Nyquist planes."""
    X, Y, Z, nyq = _freqs(grid)
    r2 = (X * X + Y * Y) * width_xy ** 2
    env = (1.0 + r2 + (Z * width_z) ** 2) ** -2.0
    phase = defocus * (X * X + Y * Y) * Z * width_xy ** 2 * width_z
    otf = env * np.exp(1j * phase)
    if cone is not None:
        otf = otf * (np.abs(Z) * width_z <= cone * np.sqrt(r2) + 1.0)
    otf[nyq] = 0.0
    otf = otf.astype(np.complex64)
    if half:
        otf = np.ascontiguousarray(otf[:, :, : int(grid.n[2]) // 2 + 1])
    return otf


def half_spectrum(otf_full: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(otf_full[:, :, : otf_full.shape[2] // 2 + 1])
