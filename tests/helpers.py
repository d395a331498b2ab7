"""Shared test helpers: float32-rounded inputs for the oracle, comparisons,
and the expected band built from the oracle's own frequency rule."""
import dataclasses

import numpy as np


def f32(x):
    return np.float64(np.float32(x))


def f32_grid(g):
    """The grid exactly as the float32 C ABI sees it."""
    return dataclasses.replace(g, spacing=tuple(float(f32(s)) for s in g.spacing),
                               origin=tuple(float(f32(s)) for s in g.origin), tau=float(f32(g.tau)))


def f32_sigma(S):
    return tuple(float(f32(s)) for s in S)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def expected_band(ref, grid, sigma):
    """Band entries (half-spectrum position, k) from the oracle's definition:
    every half-spectrum position carries the DFT frequency of its full-grid
    index and, at Nyquist positions, the alias with the Nyquist components
    negated; an entry is kept iff the oracle's band rule accepts it."""
    n0, n1, n2 = grid.n
    n2h = n2 // 2 + 1
    kx = ref.int_freqs(n0)
    ky = ref.int_freqs(n1)
    kz_full = ref.int_freqs(n2)
    ix, iy, iz = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2h), indexing="ij")
    K = np.stack([kx[ix], ky[iy], kz_full[iz]], -1).reshape(-1, 3)
    pos = ((ix * n1 + iy) * n2h + iz).reshape(-1)
    nyx = (n0 % 2 == 0) & (ix.reshape(-1) == n0 // 2)
    nyy = (n1 % 2 == 0) & (iy.reshape(-1) == n1 // 2)
    nyz = (n2 % 2 == 0) & (iz.reshape(-1) == n2 // 2)
    anyn = nyx | nyy | nyz
    K2 = K.copy()
    K2[nyx, 0] *= -1
    K2[nyy, 1] *= -1
    K2[nyz, 2] *= -1
    thr = ref.band_threshold(grid.tau)
    in1 = ref.quad_form(ref.xi_of_k(K, grid), sigma) < thr
    in2 = (ref.quad_form(ref.xi_of_k(K2, grid), sigma) < thr) & anyn
    w1 = np.where(anyn, 0.5, 1.0)
    ent_pos = np.concatenate([pos[in1], pos[in2]])
    ent_k = np.concatenate([K[in1], K2[in2]])
    ent_w = np.concatenate([w1[in1], w1[in2]])
    return ent_pos, ent_k, ent_w


def sort_entries(pos, k):
    key = np.lexsort((k[:, 2], k[:, 1], k[:, 0], pos))
    return key
