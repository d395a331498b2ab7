"""Pins of the oracle's per-triangle density weights (paper Sec. 3.3: several
surfaces or materials as a weighted sum of densities; cell-cell interfaces
as double membranes).  Surface density: each triangle's term times w_T,
normalised by sum_T w_T A_T.  Indicator density: w_T is the density jump
across the triangle (behind minus in front of its normal)."""
import numpy as np
import pytest

from oracle.reference import SURFACE, VOLUME
from workloads import meshes


def sinc(a):
    a = np.asarray(a, dtype=np.float64)
    out = np.ones_like(a)
    nz = a != 0
    out[nz] = np.sin(a[nz]) / a[nz]
    return out


def box_volume_ft(lo, hi, xi):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    L, c = hi - lo, (hi + lo) / 2
    return np.prod(L) * np.prod(sinc(xi * L / 2), axis=-1) * np.exp(-1j * xi @ c)


def box_surface_ft(lo, hi, xi):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    L, c = hi - lo, (hi + lo) / 2
    s, co = sinc(xi * L / 2), np.cos(xi * L / 2)
    t = (L[1] * L[2] * co[..., 0] * s[..., 1] * s[..., 2] + L[0] * L[2] * s[..., 0] * co[..., 1] * s[..., 2]
         + L[0] * L[1] * s[..., 0] * s[..., 1] * co[..., 2])
    return 2 * t * np.exp(-1j * xi @ c)


def densities_to_weights(side, rho, mode):
    """Volume: jump rho(back) - rho(front); surface: number of membranes."""
    r = np.concatenate([np.asarray(rho, float), [0.0]])   # index -1 -> outside
    if mode == VOLUME:
        return r[side[:, 0]] - r[side[:, 1]]
    return np.where(side[:, 1] >= 0, 2.0, 1.0)


def xis(n=30, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-4, 4, size=(n, 3))
    x[0] = 0.0
    x[1] = [1.3, 0.0, 0.0]
    return x


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_unit_weights_equal_the_unweighted_transform(ref, mode):
    V, F = meshes.icosphere(2)
    xi = xis()
    w = np.ones(len(F))
    a, b = ref.mesh_ft_raw(V, F, xi, mode), ref.mesh_ft_raw(V, F, xi, mode, w)
    assert np.array_equal(a, b)
    W = np.exp(1j * np.arange(len(xi)))
    assert np.array_equal(ref.mesh_ft_vjp_raw(V, F, xi, W, mode), ref.mesh_ft_vjp_raw(V, F, xi, W, mode, w))


def test_two_cells_of_different_density_volume_closed_form(ref):
    s = 1.7
    V, F, side = meshes.cube_foam((2, 1, 1), sub=2, size=s)
    V = V + np.array([0.3, -0.2, 0.5])
    rho = [0.7, 1.6]
    w = densities_to_weights(side, rho, VOLUME)
    xi = xis()
    lo0 = np.array([0.3, -0.2, 0.5])
    want = rho[0] * box_volume_ft(lo0, lo0 + s, xi) + rho[1] * box_volume_ft(lo0 + [s, 0, 0], lo0 + [2 * s, s, s], xi)
    got = ref.mesh_ft_raw(V, F, xi, VOLUME, w)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_double_membrane_surface_closed_form(ref):
    s = 1.3
    V, F, side = meshes.cube_foam((2, 1, 1), sub=2, size=s)
    w = densities_to_weights(side, [1, 1], SURFACE)
    xi = xis(seed=4)
    want = box_surface_ft([0, 0, 0], [s, s, s], xi) + box_surface_ft([s, 0, 0], [2 * s, s, s], xi)
    got = ref.mesh_ft_raw(V, F, xi, SURFACE, w)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    assert abs(ref.surface_area(V, F, w) - 12 * s * s) < 1e-12


def test_deformed_foam_volume_equals_sum_of_cells_by_cones(ref):
    """Eight deformed cells with random densities: the weighted divergence
    sum equals the density-weighted sum of each closed cell's transform,
    computed by the independent cone decomposition."""
    V, F, side = meshes.cube_foam((2, 2, 2), sub=2, size=1.0)
    V = meshes.foam_deform(V, np.random.default_rng(5))
    rho = np.random.default_rng(6).uniform(0.5, 1.5, size=8)
    w = densities_to_weights(side, rho, VOLUME)
    xi = xis(n=20, seed=7)
    want = np.zeros(len(xi), complex)
    for c in range(8):
        sel = (side[:, 0] == c) | (side[:, 1] == c)
        Fc = F[sel].copy()
        inward = side[sel][:, 1] == c
        Fc[inward] = Fc[inward][:, [0, 2, 1]]
        assert meshes.check_closed_oriented(Fc)
        want += rho[c] * ref.cone_volume_ft(V, Fc, xi)
    got = ref.mesh_ft_raw(V, F, xi, VOLUME, w)
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_weighted_vertex_gradient_matches_finite_differences(ref, mode):
    V, F, side = meshes.cube_foam((2, 1, 1), sub=2, size=1.0)
    V = meshes.foam_deform(V, np.random.default_rng(8))
    w = densities_to_weights(side, [0.8, 1.3], mode)
    rng = np.random.default_rng(9)
    xi = rng.normal(size=(10, 3)) * 1.5
    xi[0] = 0.0
    W = rng.normal(size=10) + 1j * rng.normal(size=10)

    def loss(Vx):
        u = ref.mesh_ft_raw(Vx, F, xi, mode, w)
        if mode == SURFACE:
            u = u / ref.surface_area(Vx, F, w)
        return float(np.real(np.sum(W * u)))

    g = ref.mesh_ft_vjp_raw(V, F, xi, W, mode, w)
    h = 1e-5
    for vi in [0, 4, 9, 13, len(V) - 1]:
        for j in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[vi, j] += h
            Vm[vi, j] -= h
            fd = (loss(Vp) - loss(Vm)) / (2 * h)
            assert abs(g[vi, j] - fd) < 1e-6 * np.abs(g).max(), (vi, j, g[vi, j], fd)
