"""Pins of the oracle's tabulated-OTF rendering (a PSF given as an array of
its transform): it reproduces the Gaussian path when tabulated from it, a
linear phase ramp (an integer-voxel shift of the PSF) rolls the image
exactly, the tables of workloads.psfs are Hermitian, and the vertex gradient
matches finite differences."""
import dataclasses

import numpy as np
import pytest

from workloads import configs, psfs


def _case(mode):
    c = configs.cfg1(mode)
    return c, dataclasses.replace(c.grid, tau=0.0)


@pytest.mark.parametrize("mode", [configs.VOLUME, configs.SURFACE])
def test_tabulated_gaussian_equals_the_gaussian_path(ref, mode):
    c, g = _case(mode)
    V = c.V.astype(np.float64)
    _, h, _ = ref.otf_and_band(g, c.sigma)
    a = ref.render(V, c.F, g, c.sigma)
    b = ref.render_otf(V, c.F, g, h)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("mode", [configs.VOLUME, configs.SURFACE])
def test_phase_ramp_rolls_the_image(ref, mode):
    c, g = _case(mode)
    V = c.V.astype(np.float64)
    otf = psfs.aberrated_otf(g, 1.0, 2.0, defocus=0.7).astype(np.complex128)
    shift = np.array([3, -2, 5])
    k = ref.full_grid_k(g)
    ramp = np.exp(-2j * np.pi * (k @ (shift / np.asarray(g.n))))
    a = ref.render_otf(V, c.F, g, otf)
    b = ref.render_otf(V, c.F, g, otf * ramp)
    assert np.abs(np.roll(a, tuple(shift), axis=(0, 1, 2)) - b).max() < 1e-12 * np.abs(a).max()


def test_tables_are_hermitian_and_the_image_is_their_real_psf(ref):
    g = configs.cfg1().grid
    otf = psfs.aberrated_otf(g, 1.0, 2.0, defocus=1.3, cone=1.5).astype(np.complex128)
    flip = np.roll(otf[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))      # otf[-k]
    assert np.array_equal(flip, np.conj(otf))
    psf = np.fft.ifftn(otf)
    assert np.abs(psf.imag).max() < 1e-12 * np.abs(psf.real).max()


@pytest.mark.parametrize("mode", [configs.VOLUME, configs.SURFACE])
def test_otf_vertex_gradient_matches_finite_differences(ref, mode):
    c, g = _case(mode)
    g = dataclasses.replace(g, tau=1e-3)
    V = c.V.astype(np.float64)
    otf = psfs.aberrated_otf(g, 1.0, 2.0, defocus=0.9, cone=1.2).astype(np.complex128)
    dI = np.random.default_rng(1).standard_normal(g.n)

    def loss(Vx):
        return float((ref.render_otf(Vx, c.F, g, otf) * dI).sum())

    dv = ref.render_otf_vjp(V, c.F, g, otf, dI)
    h = 1e-4
    for vi in [0, 40, 111]:
        for j in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[vi, j] += h
            Vm[vi, j] -= h
            fd = (loss(Vp) - loss(Vm)) / (2 * h)
            assert abs(dv[vi, j] - fd) < 1e-6 * np.abs(dv).max(), (vi, j, dv[vi, j], fd)
