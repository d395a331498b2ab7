"""Tabulated PSFs on the GPU (dm_render_otf / dm_render_otf_vjp) against the
FP64 oracle, the Gaussian path and the exact shift rule."""
import dataclasses
import sys

import numpy as np
import pytest

from helpers import f32_grid, rel_l2
from workloads import configs, psfs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_10440_amd as m
    return m


@pytest.fixture(scope="module")
def handle(dm):
    return dm.Handle(0)


def dev(x, dtype=np.float32):
    import torch
    return torch.tensor(np.ascontiguousarray(x, dtype=dtype), device="cuda:0")


def _grids():
    g1 = f32_grid(configs.cfg1().grid)
    godd = f32_grid(dataclasses.replace(configs.cfg1().grid, n=(30, 31, 33)))
    return [("32^3", g1), ("30x31x33", godd)]


@pytest.mark.parametrize("gi", [0, 1])
@pytest.mark.parametrize("mode", [configs.VOLUME, configs.SURFACE])
def test_aberrated_otf_image_and_gradient(dm, handle, ref, mode, gi):
    name, g = _grids()[gi]
    g = dataclasses.replace(g, mode=mode)
    c = configs.cfg1(mode)
    otf = psfs.aberrated_otf(g, 1.0, 2.0, defocus=0.9, cone=1.2)
    say("tabulated otf", name, "mode", mode)
    topo = handle.topology(c.F, n_verts=len(c.V))
    V64 = c.V.astype(np.float64)
    img = dm.render_otf(handle, dev(c.V), topo, dev(psfs.half_spectrum(otf), np.complex64), g).cpu().numpy()
    want = ref.render_otf(V64, c.F, g, otf.astype(np.complex128))
    G = np.random.default_rng(2).standard_normal(g.n).astype(np.float32)
    dv, img2 = dm.render_otf_vjp(handle, dev(c.V), topo, dev(psfs.half_spectrum(otf), np.complex64), g, dev(G),
                                 want_image=True)
    dvw = ref.render_otf_vjp(V64, c.F, g, otf.astype(np.complex128), G.astype(np.float64))
    e_img, e_dv = rel_l2(img, want), rel_l2(dv.cpu().numpy(), dvw)
    e_img2 = rel_l2(img2.cpu().numpy(), want)
    say("  image", e_img, "dV", e_dv, "image of the gradient call", e_img2)
    assert e_img < 1e-5 and e_dv < 1e-4 and e_img2 < 1e-5
    # the gradient call computes its image in the fused sweep: the same sums in
    # another float32 order
    assert rel_l2(img2.cpu().numpy(), img) < 1e-6


def test_tabulated_gaussian_equals_the_gaussian_path(dm, handle, ref):
    c = configs.cfg1()
    g = dataclasses.replace(f32_grid(c.grid), tau=0.0)
    _, h, _ = ref.otf_and_band(g, tuple(float(np.float32(x)) for x in c.sigma))
    topo = handle.topology(c.F, n_verts=len(c.V))
    a = dm.render(handle, dev(c.V), topo, c.sigma, g).cpu().numpy()
    b = dm.render_otf(handle, dev(c.V), topo, dev(psfs.half_spectrum(h.astype(np.complex64)), np.complex64),
                      g).cpu().numpy()
    say("tabulated Gaussian vs Gaussian path", rel_l2(b, a))
    assert rel_l2(b, a) < 1e-6


def test_phase_ramp_rolls_the_image(dm, handle, ref):
    c = configs.cfg1(configs.SURFACE)
    g = f32_grid(c.grid)
    otf = psfs.aberrated_otf(g, 1.0, 2.0, defocus=0.5).astype(np.complex128)
    shift = np.array([4, -3, 2])
    ramp = np.exp(-2j * np.pi * (ref.full_grid_k(g) @ (shift / np.asarray(g.n))))
    topo = handle.topology(c.F, n_verts=len(c.V))
    a = dm.render_otf(handle, dev(c.V), topo, dev(psfs.half_spectrum(otf), np.complex64), g).cpu().numpy()
    b = dm.render_otf(handle, dev(c.V), topo, dev(psfs.half_spectrum(otf * ramp), np.complex64), g).cpu().numpy()
    e = rel_l2(b, np.roll(a, tuple(shift), axis=(0, 1, 2)))
    say("phase ramp roll", e)
    assert e < 1e-5


def test_otf_errors(dm, handle):
    import torch
    c = configs.cfg1()
    g = c.grid
    topo = handle.topology(c.F, n_verts=len(c.V))
    bad = torch.zeros((32, 32, 32), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(ValueError):
        dm.render_otf(handle, dev(c.V), topo, bad, g)
    with pytest.raises(TypeError):
        dm.render_otf(handle, dev(c.V), topo, bad.real.contiguous(), g)
    open_F = c.F[1:]
    topo2 = handle.topology(open_F, n_verts=len(c.V))
    ok = torch.ones((32, 32, 17), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(Exception):
        dm.render_otf(handle, dev(c.V), topo2, ok, g)
