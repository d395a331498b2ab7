"""The five workloads the renderer is measured and checked on, as seeded inputs.

Each builder returns plain arrays and numbers: float32 vertices, int32 faces,
a grid (voxel counts, spacing, origin, band threshold) and a Gaussian PSF
covariance.  Nothing here evaluates the mesh transform.

Units: vertex positions, spacing and PSF standard deviations share one length
unit (voxels for the workloads stated in voxels, micrometres otherwise).  The
grid origin is the position of voxel (0,0,0); voxel centres sit at
``origin + i * spacing``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import meshes

VOLUME = 0    # indicator function of the enclosed region
SURFACE = 1   # area-normalised surface density of the paper's Sec. 4.1


@dataclasses.dataclass(frozen=True)
class Grid:
    n: tuple[int, int, int]
    spacing: tuple[float, float, float]
    origin: tuple[float, float, float] = (0.0, 0.0, 0.0)
    tau: float = 1e-3          # band: OTF value strictly above tau (0 = full spectrum)
    mode: int = VOLUME

    def with_mode(self, mode: int) -> "Grid":
        return dataclasses.replace(self, mode=mode)

    def with_tau(self, tau: float) -> "Grid":
        return dataclasses.replace(self, tau=tau)

    @property
    def centre(self) -> np.ndarray:
        return np.array(self.origin) + (np.array(self.n) - 1) / 2.0 * np.array(self.spacing)


def psf_diag(sigma_xy: float, sigma_z: float) -> tuple[float, ...]:
    """Axis-aligned Gaussian PSF as the 6-entry covariance (xx, yy, zz, xy, xz, yz)."""
    return (sigma_xy ** 2, sigma_xy ** 2, sigma_z ** 2, 0.0, 0.0, 0.0)


@dataclasses.dataclass
class Case:
    name: str
    V: np.ndarray          # float32 [n_v, 3]
    F: np.ndarray          # int32 [n_t, 3]
    grid: Grid
    sigma: tuple[float, ...]
    extra: dict = dataclasses.field(default_factory=dict)


def _f32(V) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(V, dtype=np.float32))


def _i32(F) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(F, dtype=np.int32))


def sphere_case(sub: int = 2, radius: float = 10.0, n=(32, 32, 32), spacing=(1.0, 1.0, 1.0),
                sigma_xy: float = 1.0, sigma_z: float = 2.5, tau: float = 1e-3, mode: int = VOLUME,
                name: str = "sphere") -> Case:
    g = Grid(tuple(n), tuple(float(s) for s in spacing), (0.0, 0.0, 0.0), tau, mode)
    U, F = meshes.icosphere(sub)
    V = U * radius + g.centre
    return Case(name, _f32(V), _i32(F), g, psf_diag(sigma_xy, sigma_z))


def cfg1(mode: int = VOLUME) -> Case:
    """Icosphere subdivision 2 (162 v / 320 t), radius 10 voxels, centred in 32^3,
    unit spacing; sigma_xy = 1, sigma_z = 2.5 voxels; band OTF > 1e-3."""
    return sphere_case(2, 10.0, (32, 32, 32), (1, 1, 1), 1.0, 2.5, 1e-3, mode, "cfg1")


def cfg2(mode: int = VOLUME, seed_jitter: int = 0, seed_noise: int = 1) -> Case:
    """cfg1's sphere with N(0, 0.5 voxel) vertex jitter; the target image is the
    unjittered render plus N(0, (0.02 max I)^2) noise, drawn here as a unit-normal
    field that the caller scales by 0.02 max(target)."""
    base = cfg1(mode)
    rng = np.random.default_rng(seed_jitter)
    Vj = base.V.astype(np.float64) + rng.normal(0.0, 0.5, size=base.V.shape)
    noise = np.random.default_rng(seed_noise).standard_normal(base.grid.n)
    return Case("cfg2", _f32(Vj), base.F, base.grid, base.sigma,
                {"V_target": base.V, "unit_noise": noise, "noise_frac": 0.02})


def deformed_sphere(U: np.ndarray, F: np.ndarray, radius: float, centre, rng) -> tuple[np.ndarray, np.ndarray]:
    V = meshes.sh_deform(U, radius, rng) + np.asarray(centre)
    return _f32(V), _i32(F)


def cfg3(mode: int = VOLUME, seed: int = 0) -> Case:
    """Single cell: icosphere subdivision 4 (2562 v / 5120 t) with an l <= 4 real
    spherical-harmonic radial deformation, mean radius 30 xy-voxels = 6 um;
    128 x 128 x 64 grid of 0.2 x 0.2 x 0.5 um voxels; sigma = (0.15, 0.15, 0.45) um."""
    g = Grid((128, 128, 64), (0.2, 0.2, 0.5), (0.0, 0.0, 0.0), 1e-3, mode)
    U, F = meshes.icosphere(4)
    V, F = deformed_sphere(U, F, 6.0, g.centre, np.random.default_rng(seed))
    return Case("cfg3", V, F, g, psf_diag(0.15, 0.45))


BATCH_GRIDS = ((64, 64, 64), (96, 96, 96), (128, 128, 64))
SERVE_GRIDS = ((64, 64, 64), (128, 128, 128), (256, 256, 128))


def _log_uniform_tris(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def random_cell(rng: np.random.Generator, tri_lo: int, tri_hi: int, grids, name: str,
                mode: int = VOLUME) -> Case:
    """One deformed geodesic sphere with a log-uniform triangle count in
    [tri_lo, tri_hi] (frequency round(sqrt(n_t / 20))), a grid drawn uniformly from
    ``grids`` at unit voxel spacing, radius 0.3 min(N), sigma_xy = 1 and
    sigma_z ~ U[1.5, 3] voxels."""
    nt = _log_uniform_tris(rng, tri_lo, tri_hi)
    freq = max(1, int(round(math.sqrt(nt / 20.0))))
    n = tuple(grids[int(rng.integers(len(grids)))])
    g = Grid(n, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), 1e-3, mode)
    U, F = meshes.geodesic_sphere(freq)
    V, F = deformed_sphere(U, F, 0.3 * min(n), g.centre, rng)
    sz = float(rng.uniform(1.5, 3.0))
    return Case(name, V, F, g, psf_diag(1.0, sz), {"geodesic_freq": freq})


def cfg4(seed: int = 0, count: int = 64, mode: int = VOLUME) -> list[Case]:
    """Batched: 64 independent deformed spheres, n_t log-uniform in [1k, 20k],
    grids from {64^3, 96^3, 128x128x64}, sigma_z ~ U[1.5, 3] voxels."""
    rng = np.random.default_rng(seed)
    return [random_cell(rng, 1000, 20000, BATCH_GRIDS, f"cfg4_{i}", mode) for i in range(count)]


def cfg5_trace(seed: int = 0, count: int = 2000, rate: float = 200.0, mode: int = VOLUME,
               warmup: int = 100):
    """Serving: Poisson arrivals at ``rate`` req/s; each request is a deformed
    sphere with n_t log-uniform in [500, 40k] and a grid from
    {64^3, 128^3, 256x256x128}.  Returns (arrival_times_s, cases); the first
    ``warmup`` requests are warm-up."""
    rng = np.random.default_rng(seed)
    total = count + warmup
    gaps = rng.exponential(1.0 / rate, size=total)
    t = np.cumsum(gaps)
    cases = [random_cell(rng, 500, 40000, SERVE_GRIDS, f"cfg5_{i}", mode) for i in range(total)]
    return t, cases


def cfg5_pooled(seed: int = 0, count: int = 200, rate: float = 200.0, pool: int = 32, warmup: int = 20):
    """cfg5 with resident meshes: a pool of ``pool`` cells drawn from the cfg5
    distribution (each with its own grid and PSF); request i uses cell
    idx[i] (uniform over the pool), arrivals Poisson at ``rate``.  Returns
    (pool_cases, arrival_times_s [count], idx [count], warmup_idx [warmup])."""
    rng = np.random.default_rng(seed)
    cases = [random_cell(rng, 500, 40000, SERVE_GRIDS, f"cfg5_pool_{i}") for i in range(pool)]
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    idx = rng.integers(pool, size=count)
    widx = rng.integers(pool, size=warmup)
    return cases, t, idx, widx


def box_case(lo=(10.25, 11.5, 9.75), hi=(19.5, 17.25, 23.0), n=(32, 32, 32), mode: int = VOLUME,
             sigma_xy: float = 1.0, sigma_z: float = 2.0, tau: float = 1e-3) -> Case:
    """Axis-aligned box: every edge is parallel to a grid axis, so on the
    coordinate planes of frequency space two or three vertex phases coincide
    exactly (the degenerate cases of the triangle transform)."""
    V, F = meshes.box_mesh(lo, hi)
    g = Grid(tuple(n), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), tau, mode)
    return Case("box", _f32(V), _i32(F), g, psf_diag(sigma_xy, sigma_z))


def foam_weights(side: np.ndarray, rho, mode: int) -> np.ndarray:
    """Per-face density weights of a cell cluster from the cells on both
    sides of every face (``meshes.cube_foam``): surface density, 2 on walls
    between two cells (double membranes) and 1 on the outside; indicator
    density, the jump rho(behind) - rho(in front), the outside at 0."""
    if mode == SURFACE:
        return np.where(side[:, 1] >= 0, 2.0, 1.0).astype(np.float32)
    r = np.concatenate([np.asarray(rho, dtype=np.float64), [0.0]])
    return (r[side[:, 0]] - r[side[:, 1]]).astype(np.float32)


def foam_case(mode: int = SURFACE, seed: int = 0, cells=(2, 2, 2), sub: int = 8, n=(128, 128, 64),
              spacing=(0.2, 0.2, 0.5), block: float = 12.0, sigma=(0.15, 0.45), tau: float = 1e-3,
              name: str = "foam") -> Case:
    """A cluster of cells sharing their walls (non-manifold, multimaterial):
    a cube foam of ``cells`` box cells, every face split into sub x sub pairs
    of triangles, rounded and wobbled smoothly, scaled to a block of
    ``block`` length units and centred in the grid.  Defaults: 8 cells,
    4608 triangles, in the single-cell grid (128 x 128 x 64 of 0.2 x 0.2 x
    0.5 um, sigma (0.15, 0.15, 0.45) um).  ``extra``: the per-face weights for
    ``mode`` (walls doubled for the surface density; for the indicator density
    cell densities drawn from U[0.5, 1.5]), the face sides and the densities."""
    rng = np.random.default_rng(seed)
    g = Grid(tuple(n), tuple(float(s) for s in spacing), (0.0, 0.0, 0.0), tau, mode)
    V, F, side = meshes.cube_foam(cells, sub=sub, size=1.0)
    V = meshes.foam_deform(V, rng)
    V = (V - 0.5 * (V.min(0) + V.max(0))) * (block / float(max(cells))) + g.centre
    rho = rng.uniform(0.5, 1.5, size=int(np.prod(cells)))
    w = foam_weights(side, rho, mode)
    return Case(name, _f32(V), _i32(F), g, psf_diag(*sigma), {"tri_w": w, "side": side, "rho": rho})
